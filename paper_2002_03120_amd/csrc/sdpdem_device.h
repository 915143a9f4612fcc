// sdpdem_device.h -- device helpers shared by the kernel translation units.
#pragma once
#include <cmath>

#include "sdpdem_internal.h"

namespace sdpdem {

static constexpr int BS = 256;
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

// Lucy kernel with support H (Eq. kernel), double precision
__device__ __forceinline__ double lucy_w(double r, double H) {
  if (r >= H) return 0.0;
  double q = r / H;
  double om = 1.0 - q;
  return 105.0 / (16.0 * PI * H * H * H) * (1.0 + 3.0 * q) * om * om * om;
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
    uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
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

// nine standard normals of the unordered pair {a, b} at a step; the tenth
// Box-Muller output is not used
__device__ __forceinline__ void pair_normals(uint32_t a, uint32_t b, uint32_t step, uint32_t k0,
                                             uint32_t k1, float z[9]) {
  uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
  float u[12];
#pragma unroll
  for (uint32_t blk = 0; blk < 3; ++blk) {
    uint32_t c0 = lo, c1 = hi, c2 = step, c3 = blk;
    philox10(c0, c1, c2, c3, k0, k1);
    u[4 * blk + 0] = u01(c0);
    u[4 * blk + 1] = u01(c1);
    u[4 * blk + 2] = u01(c2);
    u[4 * blk + 3] = u01(c3);
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    float rad = sqrtf(-2.0f * logf(u[2 * m]));
    float sn, cs;
    sincospif(2.0f * u[2 * m + 1], &sn, &cs);
    if (2 * m < 9) z[2 * m] = rad * cs;
    if (2 * m + 1 < 9) z[2 * m + 1] = rad * sn;
  }
}


}  // namespace sdpdem
