// sdpdem_device.h -- device helpers shared by the kernel translation units.
#pragma once
#include <cmath>

#include "sdpdem_internal.h"

namespace sdpdem {

static constexpr double PI = 3.14159265358979323846;

inline int nblocks(size_t n, int bs = BS) {
  size_t b = (n + bs - 1) / bs;
  b = (b + 7) / 8 * 8;  // a multiple of the 8 XCDs
  return (int)(b > 0 ? b : 8);
}

// Block index -> particle chunk, contiguous per XCD.
__device__ __forceinline__ int xcd_tid() {
  unsigned nb = gridDim.x, b = blockIdx.x;
  unsigned lb = (nb % 8u == 0u) ? (b % 8u) * (nb / 8u) + (b / 8u) : b;
  return (int)(lb * blockDim.x + threadIdx.x);
}

// Global wavefront index with blocks taken in XCD order: consecutive
// wavefronts (neighbouring spheres in cell order) share an XCD and its L2.
__device__ __forceinline__ int xcd_wave() {
  unsigned nb = gridDim.x, b = blockIdx.x;
  unsigned lb = (nb % 8u == 0u) ? (b % 8u) * (nb / 8u) + (b / 8u) : b;
  return (int)((lb * blockDim.x + threadIdx.x) >> 6);
}

// The launch-table entry of this block.  Block b runs on XCD b % 8 as that
// XCD's (b / 8)-th block; the XCD takes chunks x, x + 8, x + 16, ... of
// blk_per consecutive entries: a chunk's particles (and most of their
// neighbours) share an L2.  With many chunks per XCD each XCD's share
// spreads over the whole sorted order, so that uneven work (outer walls
// in one region of the box) lands on every XCD alike; with one chunk per
// XCD each takes one contiguous eighth.
template <bool ACT = false>
__device__ __forceinline__ unsigned logical_block(const Dev& d) {
  const unsigned b = blockIdx.x, per = (unsigned)(ACT ? d.ablk_per : d.blk_per);
  const unsigned k = b / 8u;
  return ((k / per) * 8u + b % 8u) * per + k % per;
}

// Launch block -> (box, first sorted particle): the box is uniform over a
// block, so its constants are scalar loads.  ACT: the table of the boxes'
// active parts (launched with nablk blocks); its last block of a box may
// reach into the box's outer walls, which every kernel skips or gives
// their fixed values.
template <bool ACT = false>
__device__ __forceinline__ int blk_box(const Dev& d, int& i) {
  const unsigned lb = logical_block<ACT>(d);
  const int2 e = ACT ? d.ablk[lb] : d.blk[lb];
  i = e.y + (int)threadIdx.x;
  return __builtin_amdgcn_readfirstlane(e.x);
}

__device__ __forceinline__ double min_img(double d, int per, double L, double halfL) {
  if (per) {
    if (d > halfL)
      d = d - L;
    else if (d < -halfL)
      d = d + L;
  }
  return d;
}

// r^2 = (dx*dx + dy*dy) + dz*dz with every product and sum rounded (no
// contraction), so that neighbour membership is the same bit for bit as a
// plain double-precision evaluation of the definition.
__device__ __forceinline__ double r2_exact(double a, double b, double c) {
#pragma clang fp contract(off)
  double t = a * a;
  double u = b * b;
  double v = c * c;
  return (t + u) + v;
}

// Minimum-image separation in box B, in place; returns k_z, the number of
// boxes by which the partner's image is displaced along z (its velocity is
// then v + k_z le_jump e_x).  With Lees-Edwards shear the z image is taken
// first, its x offset applied, and x wrapped; otherwise axis by axis.
__device__ __forceinline__ Geo geo_of(const BoxD& B) {
  Geo g;
  for (int a = 0; a < 3; ++a) {
    g.L[a] = B.L[a];
    g.halfL[a] = B.halfL[a];
    g.lim[a] = B.per[a] ? B.halfL[a] : __builtin_inf();
    g.per[a] = B.per[a];
  }
  g.inv_Lx = 1.0 / B.L[0];
  g.le_shift = B.le_shift;
  g.le_jump = B.le_jump;
  g.le = B.le;
  return g;
}

__device__ __forceinline__ int min_img_box(const Geo& B, double& ex, double& ey, double& ez) {
#pragma clang fp contract(off)
  int kz = 0;
  if (B.per[2]) {
    if (ez > B.halfL[2]) {
      ez = ez - B.L[2];
      kz = 1;
    } else if (ez < -B.halfL[2]) {
      ez = ez + B.L[2];
      kz = -1;
    }
  }
  if (B.le) {
    // rint(ex / L) with a multiply: it can differ from the quotient's only
    // where ex / L sits within an ulp of a half-integer, where both images
    // are equally near (and L/2 is at least 1.5 cells, beyond the SDPD and
    // coupling cut-offs)
    ex = ex - B.le_shift * (double)kz;
    ex = ex - B.L[0] * rint(ex * B.inv_Lx);
  } else {
    ex = min_img(ex, B.per[0], B.L[0], B.halfL[0]);
  }
  ey = min_img(ey, B.per[1], B.L[1], B.halfL[1]);
  return kz;
}

// min_img_box with a shortcut.  Within half the box on every periodic axis
// a separation is already its minimum image, with no z image: min_img_box
// would return it bit for bit (its x rint at exactly half the box could
// pick the other, equally near image, which lies beyond every cut-off).
// That holds for all pairs away from the periodic seams, and three
// compares replace the image arithmetic there; boxes without a periodic
// axis skip both (a test uniform over the launch block).  Used where the
// image arithmetic costs issue slots (the searches and filters, the
// thermal pair kernel); in the gather-bound deterministic pair loop the
// plain form schedules its loads better.
__device__ __forceinline__ int min_img_fast(const Geo& B, double& ex, double& ey, double& ez) {
  if (!(B.per[0] | B.per[1] | B.per[2])) return 0;
  if (fabs(ex) <= B.lim[0] && fabs(ey) <= B.lim[1] && fabs(ez) <= B.lim[2]) return 0;
  return min_img_box(B, ex, ey, ez);
}

__device__ __forceinline__ int cell_coord(double x, const Grid& g, int a, int* oob) {
  double f = floor((x - g.lo[a]) * g.inv_cs[a]);
  int n = g.nc[a];
  if (g.per[a]) {
    f = f - (double)n * floor(f / (double)n);
    if (!(f >= 0.0 && f < (double)n)) {
      *oob = 1;
      return 0;
    }
    return (int)f;
  }
  if (!(f >= 0.0)) {
    *oob = 1;
    return 0;
  }
  if (f >= (double)n) {
    *oob = 1;
    return n - 1;
  }
  return (int)f;
}

__device__ __forceinline__ int cell_index(const Grid& g, int cx, int cy, int cz) {
  return (cz * g.nc[1] + cy) * g.nc[0] + cx;
}

// wrap (periodic) or reject (wall) a neighbour cell coordinate
__device__ __forceinline__ bool wrap_axis(int& c, int n, int per) {
  if (c < 0) {
    if (!per) return false;
    c += n;
  } else if (c >= n) {
    if (!per) return false;
    c -= n;
  }
  return true;
}

// square root of x >= 0 from the hardware reciprocal square root and one
// Newton correction of the residual x - s^2 (relative error far below the
// FP64 density tolerance; exact 0 for x = 0)
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double s = x * y;
  const double e = __builtin_fma(-s, s, x);
  const double r = __builtin_fma(e, 0.5 * y, s);
  return x > 0.0 ? r : 0.0;
}

// one 64-byte pair record (four 16-byte loads from one cache line)
__device__ __forceinline__ PR load_pr(const PR* base, int j) { return base[j]; }

// The cells that can hold partners within R of a point (px, py, pz) in
// cell cc of a box's grid G, searched over the (2k+1)^2 rows (z, y) around
// cc (all rows of an axis when the stencil would wrap onto itself).  A row
// whose slab lies R or more away from the point in y and z is empty; in
// the others only the x cells within sqrt(R^2 - d^2) of the point's x (d
// its distance to the slab) are taken, at most the 2k+1 cells around cc.
// Rows seen through a Lees-Edwards z face are centred on the shifted x
// coordinate; when the stencil wraps onto itself along z under shear every
// x cell is taken.  Row r holds at most two runs of consecutive x cells,
// [a0, a1) and [b0, b1) in global keys (off = the box's cell offset);
// empty runs have a0 == a1.  The x range carries a relative margin of 1e-9
// so that the distance test, not the range, decides.
struct StencilShape {
  int zlo, zn, ylo, yn;
  bool zall, yall;
};

__device__ __forceinline__ StencilShape stencil_shape(const Grid& G, const int cc[3], int k) {
  StencilShape sh;
  sh.zall = G.per[2] && 2 * k + 1 > G.nc[2];
  sh.yall = G.per[1] && 2 * k + 1 > G.nc[1];
  sh.zlo = sh.zall ? 0 : cc[2] - k;
  sh.zn = sh.zall ? G.nc[2] : 2 * k + 1;
  sh.ylo = sh.yall ? 0 : cc[1] - k;
  sh.yn = sh.yall ? G.nc[1] : 2 * k + 1;
  return sh;
}

// cells each way that hold every point within H of a cell's points
__device__ __forceinline__ int reach_cells(const Grid& g, double H) {
  int k = 1;
  for (int a = 0; a < 3; ++a) k = max(k, (int)ceil(H * g.inv_cs[a] * (1.0 + 1e-9)));
  return k;
}

// distance of x to the slab [lo, lo + cs)
__device__ __forceinline__ double slab_dist(double x, double lo, double cs) {
  return fmax(0.0, fmax(lo - x, x - (lo + cs)));
}

// the row at unwrapped z and y cell indices (zu, yu)
template <bool PRUNE>
__device__ __forceinline__ void stencil_row_zy(const Geo& B, const Grid& G, int off, double px,
                                               double py, double pz, double R, const int cc[3],
                                               int k, const StencilShape& sh, int zu, int yu,
                                               int& a0, int& a1, int& b0, int& b1) {
  a0 = a1 = b0 = b1 = 0;
  const int nx = G.nc[0], ny = G.nc[1], nz = G.nc[2];
  int z = zu, y = yu, wz = 0;
  if (z < 0) {
    if (!G.per[2]) return;
    z += nz;
    wz = -1;
  } else if (z >= nz) {
    if (!G.per[2]) return;
    z -= nz;
    wz = 1;
  }
  if (y < 0) {
    if (!G.per[1]) return;
    y += ny;
  } else if (y >= ny) {
    if (!G.per[1]) return;
    y -= ny;
  }
  // reach in x from the distance to the row's slab (unwrapped coordinates)
  double d2 = 0.0;
  if (PRUNE && !sh.zall) {
    const double dz = slab_dist(pz, G.lo[2] + (double)zu * G.cs[2], G.cs[2]);
    d2 += dz * dz;
  }
  if (PRUNE && !sh.yall) {
    const double dy = slab_dist(py, G.lo[1] + (double)yu * G.cs[1], G.cs[1]);
    d2 += dy * dy;
  }
  if (PRUNE && d2 >= R * R) return;
  const double rx = PRUNE ? sqrt(R * R - d2) * (1.0 + 1e-9) + 1e-9 * G.cs[0]
                          : (double)(k + 1) * G.cs[0];
  int x0, xn;
  if (B.le && sh.zall) {
    x0 = 0;
    xn = nx;
  } else {
    // candidates sit around x - k_z delta (k_z = wz, 0 off the sheared faces)
    const double xc = (B.le && wz != 0) ? px - (double)wz * B.le_shift : px;
    int xa, xb;
    if (!PRUNE && !(B.le && wz != 0)) {  // the plain stencil
      xa = cc[0] - k;
      xb = cc[0] + k;
    } else {
      xa = (int)floor((xc - rx - G.lo[0]) * G.inv_cs[0]);
      xb = (int)floor((xc + rx - G.lo[0]) * G.inv_cs[0]);
      if (!(B.le && wz != 0)) {  // never beyond the plain stencil
        xa = max(xa, cc[0] - k);
        xb = min(xb, cc[0] + k);
      }
    }
    x0 = xa;
    xn = xb - xa + 1;
    if (xn <= 0) return;
    if (G.per[0]) {
      if (xn >= nx) {
        x0 = 0;
        xn = nx;
      } else {
        // x0 lies within two box lengths of the box (a sheared image row
        // starts at most one length away): wrap by additions, which cost a
        // fraction of an integer modulo; the modulo stays for anything else
        if (x0 < 0) x0 += nx;
        if (x0 < 0) x0 += nx;
        if (x0 >= nx) x0 -= nx;
        if (x0 >= nx) x0 -= nx;
        if (x0 < 0 || x0 >= nx) x0 = ((x0 % nx) + nx) % nx;
      }
    }
  }
  const int rowkey = off + (z * ny + y) * nx;
  if (G.per[0] && xn >= nx) {
    a0 = rowkey;
    a1 = rowkey + nx;
  } else if (!G.per[0]) {
    int lo = max(x0, 0), hi = min(x0 + xn - 1, nx - 1);
    if (lo <= hi) {
      a0 = rowkey + lo;
      a1 = rowkey + hi + 1;
    }
  } else {
    int lo = x0, hi = x0 + xn - 1;  // 0 <= lo < nx: at most one wrap
    if (hi >= nx) {
      a0 = rowkey + lo;
      a1 = rowkey + nx;
      b0 = rowkey;
      b1 = rowkey + hi - nx + 1;
    } else {
      a0 = rowkey + lo;
      a1 = rowkey + hi + 1;
    }
  }
}

// row r of the stencil, z-major
template <bool PRUNE>
__device__ __forceinline__ void stencil_row(const Geo& B, const Grid& G, int off, double px,
                                            double py, double pz, double R, const int cc[3],
                                            int k, const StencilShape& sh, int r, int& a0,
                                            int& a1, int& b0, int& b1) {
  stencil_row_zy<PRUNE>(B, G, off, px, py, pz, R, cc, k, sh, sh.zlo + r / sh.yn,
                        sh.ylo + r % sh.yn, a0, a1, b0, b1);
}

// the same cells as fn(first_key, end_key) over the runs, in row order;
// PRUNE = false keeps the whole 2k+1 cells of every row (one thread per
// particle: lanes of a cell then walk the same runs in step)
template <bool PRUNE, class Fn>
__device__ __forceinline__ void for_stencil(const Geo& B, const Grid& G, int off, double px,
                                            double py, double pz, double R, const int cc[3],
                                            int k, Fn&& fn) {
  const StencilShape sh = stencil_shape(G, cc, k);
  for (int zi = 0; zi < sh.zn; ++zi)
    for (int yi = 0; yi < sh.yn; ++yi) {
      int a0, a1, b0, b1;
      stencil_row_zy<PRUNE>(B, G, off, px, py, pz, R, cc, k, sh, sh.zlo + zi, sh.ylo + yi, a0,
                            a1, b0, b1);
      if (a1 > a0) fn(a0, a1);
      if (b1 > b0) fn(b0, b1);
    }
}

// The rows of for_stencil<true> for one thread, with the row geometry in
// single precision on coordinates relative to the point's own cell (so
// their magnitude stays below a few cells): the z distance is formed once
// per z row, rows are walked z-major without an integer division, and the
// x reach takes one FP32 square root.  Every bound carries a relative
// margin of 1e-5 of a cell, far above the FP32 rounding of these small
// numbers, so the runs may hold a few extra cells but never miss one; the
// distance test in FP64 decides.  Sheared boxes (measured: the generic
// rows are faster there), stencils that wrap onto themselves and points
// outside their cell take the generic rows.
template <class Fn>
__device__ __forceinline__ void for_stencil_pruned(const Geo& B, const Grid& G, int off, double px,
                                                   double py, double pz, double R,
                                                   const int cc[3], int k, Fn&& fn) {
  const double fxd = px - (G.lo[0] + (double)cc[0] * G.cs[0]);
  const double fyd = py - (G.lo[1] + (double)cc[1] * G.cs[1]);
  const double fzd = pz - (G.lo[2] + (double)cc[2] * G.cs[2]);
  const int nx = G.nc[0], ny = G.nc[1], nz = G.nc[2];
  const bool plain = !B.le && !(G.per[2] && 2 * k + 1 > nz) && !(G.per[1] && 2 * k + 1 > ny) &&
                     fxd > -G.cs[0] && fxd < 2.0 * G.cs[0] && fyd > -G.cs[1] &&
                     fyd < 2.0 * G.cs[1] && fzd > -G.cs[2] && fzd < 2.0 * G.cs[2];
  if (!plain) {
    for_stencil<true>(B, G, off, px, py, pz, R, cc, k, fn);
    return;
  }
  const float fx = (float)fxd, fy = (float)fyd, fz = (float)fzd;
  const float csx = (float)G.cs[0], csy = (float)G.cs[1], csz = (float)G.cs[2];
  const float icx = (float)G.inv_cs[0];
  const float R2 = (float)(R * R) * (1.0f + 1e-5f);
  const float mx = 1e-5f * csx;
  for (int dz = -k; dz <= k; ++dz) {
    int z = cc[2] + dz;
    if (z < 0 || z >= nz) {
      if (!G.per[2]) continue;
      z += z < 0 ? nz : -nz;
    }
    const float sz = fmaxf(0.0f, fmaxf((float)dz * csz - fz, fz - (float)(dz + 1) * csz));
    const float z2 = sz * sz;
    if (z2 >= R2) continue;
    for (int dy = -k; dy <= k; ++dy) {
      int y = cc[1] + dy;
      if (y < 0 || y >= ny) {
        if (!G.per[1]) continue;
        y += y < 0 ? ny : -ny;
      }
      const float sy = fmaxf(0.0f, fmaxf((float)dy * csy - fy, fy - (float)(dy + 1) * csy));
      const float d2 = z2 + sy * sy;
      if (d2 >= R2) continue;
      const float rx = sqrtf(R2 - d2) * (1.0f + 1e-5f) + mx;
      const int xa = max(cc[0] + (int)floorf((fx - rx) * icx), cc[0] - k);
      const int xb = min(cc[0] + (int)floorf((fx + rx) * icx), cc[0] + k);
      if (xb < xa) continue;
      const int rowkey = off + (z * ny + y) * nx;
      if (!G.per[0]) {
        const int lo = max(xa, 0), hi = min(xb, nx - 1);
        if (lo <= hi) fn(rowkey + lo, rowkey + hi + 1);
      } else if (xb - xa + 1 >= nx) {
        fn(rowkey, rowkey + nx);
      } else {
        // xa (within k cells of the row) into [0, nx) without a division
        const int lo = xa < 0 ? xa + nx : (xa >= nx ? xa - nx : xa);
        const int hi = lo + (xb - xa);  // at most one wrap
        if (hi >= nx) {
          fn(rowkey + lo, rowkey + nx);
          fn(rowkey, rowkey + hi - nx + 1);
        } else {
          fn(rowkey + lo, rowkey + hi + 1);
        }
      }
    }
  }
}

// Block-wide exclusive scan of one int per thread (wave64 shuffles + LDS).
__device__ inline int block_exclusive_scan(int v, int* lds, int* total) {
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < BS / 64; ++w) {
      int t = lds[w];
      lds[w] = acc;
      acc += t;
    }
    lds[BS / 64] = acc;
  }
  __syncthreads();
  int res = x - v + lds[wid];
  *total = lds[BS / 64];
  __syncthreads();
  return res;
}

// Philox4x32-10 (Salmon et al., SC'11): two 32x32 -> 64-bit products per
// round with the published multipliers, Weyl key increments between rounds.
__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32 x 32 -> 64-bit product in one multiply (both halves)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ float u01(uint32_t x) {
  return (float)((x >> 8) + 1u) * 5.9604644775390625e-8f;  // (0, 1], exact
}

// four standard normals of the unordered pair {a, b} at a step (one Philox
// block, Box-Muller on two pairs of uniforms): three across e_ij and one
// along it, the thermal force of Eq. FijT in its pair frame
__device__ __forceinline__ void pair_normals(uint32_t a, uint32_t b, uint32_t step, uint32_t k0,
                                             uint32_t k1, float z[4]) {
  uint32_t c0 = a < b ? a : b, c1 = a < b ? b : a, c2 = step, c3 = 0u;
  philox10(c0, c1, c2, c3, k0, k1);
  const float u[4] = {u01(c0), u01(c1), u01(c2), u01(c3)};
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    float rad = sqrtf(-2.0f * logf(u[2 * m]));
    // sin and cos of 2 pi u by the hardware units, whose argument is in
    // revolutions (largest error 1.3e-7 over every u this generator makes)
    const float cs = __builtin_amdgcn_cosf(u[2 * m + 1]), sn = __builtin_amdgcn_sinf(u[2 * m + 1]);
    z[2 * m] = rad * cs;
    z[2 * m + 1] = rad * sn;
  }
}


}  // namespace sdpdem
