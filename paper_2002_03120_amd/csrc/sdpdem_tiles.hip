// sdpdem_tiles.hip -- the neighbour kernels, staged through LDS by brick.
//
// The main grid keys its cells brick-major (4x4x4-cell bricks ranked along
// a Morton curve).  One workgroup takes one brick: it loads the particles
// of the brick's 6x6x6-cell footprint (the brick and one cell around it)
// into LDS, in footprint-cell order, and every particle of the brick finds
// its 27 neighbour cells as nine contiguous slot ranges of that tile.  The
// neighbour lists hold these 16-bit footprint slots; the smoothing and
// pair-force kernels rebuild the same footprint (same cell starts) and
// gather neighbour records from LDS instead of scattered global lines.
//
// A brick whose footprint exceeds a kernel's tile capacity is appended to
// an overflow list and processed afterwards by the same code instantiated
// with GLOBAL = true, which reads the footprint from global memory; the
// LDS instantiation carries no fallback path at all.
#include "sdpdem_device.h"

namespace sdpdem {

static constexpr int FP = 216;  // footprint cells, x fastest

struct TileHeader {
  int foff[FP + 1];  // first slot of each footprint cell; foff[FP] = total
  int fstart[FP];    // first sorted index of each footprint cell
  int scan[BS / 64 + 1];
};

// Footprint of the brick at Morton rank `rank`; returns the brick's own
// particle range.  Every thread of the block must call it.
__device__ __forceinline__ void tile_setup(const Dev& d, int rank, TileHeader& th, int bc[3],
                                           int& own_b, int& own_e) {
  own_b = d.cstart[rank * 64];
  own_e = d.cstart[rank * 64 + 64];
  const int lin = d.brick_of_rank[rank];
  bc[0] = lin % d.g.nb[0];
  bc[1] = (lin / d.g.nb[0]) % d.g.nb[1];
  bc[2] = lin / (d.g.nb[0] * d.g.nb[1]);
  const int t = threadIdx.x;
  int cnt = 0, st = 0;
  if (t < FP) {
    int x = 4 * bc[0] - 1 + t % 6;
    int y = 4 * bc[1] - 1 + (t / 6) % 6;
    int z = 4 * bc[2] - 1 + t / 36;
    if (wrap_axis(x, d.g.nc[0], d.g.per[0]) && wrap_axis(y, d.g.nc[1], d.g.per[1]) &&
        wrap_axis(z, d.g.nc[2], d.g.per[2])) {
      int key = cell_index(d.g, x, y, z);
      st = d.cstart[key];
      cnt = d.cstart[key + 1] - st;
    }
  }
  int tot;
  int ex = block_exclusive_scan(cnt, th.scan, &tot);
  if (t < FP) {
    th.foff[t] = ex;
    th.fstart[t] = st;
  }
  if (t == 0) th.foff[FP] = tot;
  __syncthreads();
}

// sorted index of footprint slot q (q < total)
__device__ __forceinline__ int slot_to_index(const TileHeader& th, int q) {
  int lo = 0, hi = FP;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (th.foff[mid] <= q)
      lo = mid;
    else
      hi = mid;
  }
  return th.fstart[lo] + (q - th.foff[lo]);
}

// footprint cell of the local cell coordinate, first of a row of three
__device__ __forceinline__ int row_cell(int lx, int ly, int lz, int dy, int dz) {
  return ((lz + 1 + dz) * 6 + (ly + 1 + dy)) * 6 + lx;
}

// Bricks go to the XCDs round-robin (block b runs on XCD b % 8): the
// particles are unevenly spread over the Morton range of the bricks, and
// contiguous chunks per XCD would leave most of the work to a few of them.
static inline int brick_blocks(int nbricks) { return nbricks > 0 ? nbricks : 1; }
static constexpr int OVF_BLOCKS = 512;  // persistent blocks of the overflow pass

// Bricks for one block: the LDS instantiation takes its own brick and
// defers it when the footprint does not fit; the global one walks the
// overflow list.  `body(rank)` runs with the tile header set up.
template <bool GLOBAL, class Body>
__device__ __forceinline__ void for_bricks(const Dev& d, TileHeader& th, int cap, int* ovf_list,
                                           int* ovf_cnt, Body&& body) {
  if (!GLOBAL) {
    const int rank = blockIdx.x;
    if (rank >= d.g.nbricks) return;
    // empty bricks leave before any footprint work
    if (d.cstart[rank * 64] == d.cstart[rank * 64 + 64]) return;
    int bc[3], own_b, own_e;
    tile_setup(d, rank, th, bc, own_b, own_e);
    if (th.foff[FP] > cap) {
      if (threadIdx.x == 0) ovf_list[atomicAdd(ovf_cnt, 1)] = rank;
      return;
    }
    body(bc, own_b, own_e);
  } else {
    const int n = *ovf_cnt;
    for (int e = blockIdx.x; e < n; e += gridDim.x) {
      int bc[3], own_b, own_e;
      tile_setup(d, ovf_list[e], th, bc, own_b, own_e);
      body(bc, own_b, own_e);
      __syncthreads();  // the header is rewritten for the next brick
    }
  }
}

// ---------------------------------------------------------------------------
// (a2)+(a3) neighbour sets {j : r_ij^2 < h^2} (double precision, no
// contraction) and the density summation (Eq. compdens) with the equation
// of state (Eq. prtcpres) and the free-surface clamp.

static constexpr int CAP_BUILD = 1280;

template <bool GLOBAL>
__global__ __launch_bounds__(BS) void k_build_tiles(Dev d, int* ovf_list, int* ovf_cnt) {
  __shared__ TileHeader th;
  __shared__ double X[GLOBAL ? 1 : CAP_BUILD], Y[GLOBAL ? 1 : CAP_BUILD],
      Z[GLOBAL ? 1 : CAP_BUILD];
  for_bricks<GLOBAL>(d, th, CAP_BUILD, ovf_list, ovf_cnt, [&](const int* bc, int own_b,
                                                             int own_e) {
    const int tot = th.foff[FP];
    if (!GLOBAL) {
      for (int q = threadIdx.x; q < tot; q += BS) {
        D4 p = d.pos[slot_to_index(th, q)];
        X[q] = p.x;
        Y[q] = p.y;
        Z[q] = p.z;
      }
      __syncthreads();
    }
    auto slot_pos = [&](int q, double& x, double& y, double& z) {
      if (GLOBAL) {
        D4 p = d.pos[slot_to_index(th, q)];
        x = p.x;
        y = p.y;
        z = p.z;
      } else {
        x = X[q];
        y = Y[q];
        z = Z[q];
      }
    };
    const double h2 = d.h2, inv_h = 1.0 / d.h;
    const size_t np = (size_t)d.npad;
    for (int i = own_b + threadIdx.x; i < own_e; i += BS) {
      if (d.type[i] == T_OUTER) {
        d.nbr_cnt[i] = 0;
        d.rho[i] = d.rho0;
        d.p[i] = d.p_ref;
        continue;
      }
      const D4 pi = d.pos[i];
      int oob = 0;
      const int lx = cell_coord(pi.x, d.g, 0, &oob) - 4 * bc[0];
      const int ly = cell_coord(pi.y, d.g, 1, &oob) - 4 * bc[1];
      const int lz = cell_coord(pi.z, d.g, 2, &oob) - 4 * bc[2];
      const int fself = row_cell(lx, ly, lz, 0, 0) + 1;
      const int qself = th.foff[fself] + (i - th.fstart[fself]);
      int cnt = 0;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
          const int f0 = row_cell(lx, ly, lz, dy, dz);
          const int qb = th.foff[f0], qe = th.foff[f0 + 3];
          for (int q = qb; q < qe; ++q) {
            if (q == qself) continue;
            double xj, yj, zj;
            slot_pos(q, xj, yj, zj);
            double ex = min_img(pi.x - xj, d.per[0], d.L[0], d.halfL[0]);
            double ey = min_img(pi.y - yj, d.per[1], d.L[1], d.halfL[1]);
            double ez = min_img(pi.z - zj, d.per[2], d.L[2], d.halfL[2]);
            if (r2_exact(ex, ey, ez) < h2) {
              if (q > 65535) {  // slot does not fit the 16-bit list entry
                atomicOr(d.status, ST_NBR_OVERFLOW);
                continue;
              }
              if (cnt < d.maxn) d.nbr16[(size_t)cnt * np + i] = (uint16_t)q;
              ++cnt;
            }
          }
        }
      if (cnt > d.maxn) {
        atomicOr(d.status, ST_NBR_OVERFLOW);
        cnt = d.maxn;
      }
      d.nbr_cnt[i] = cnt;
      // density over the found neighbours, in a loop of its own so that the
      // kernel evaluation does not run under the divergent candidate test
      double acc = d.W0;
      for (int k = 0; k < cnt; ++k) {
        double xj, yj, zj;
        slot_pos(d.nbr16[(size_t)k * np + i], xj, yj, zj);
        double ex = min_img(pi.x - xj, d.per[0], d.L[0], d.halfL[0]);
        double ey = min_img(pi.y - yj, d.per[1], d.L[1], d.halfL[1]);
        double ez = min_img(pi.z - zj, d.per[2], d.L[2], d.halfL[2]);
        double qq = sqrt(ex * ex + ey * ey + ez * ez) * inv_h;
        double om = 1.0 - qq;
        acc += d.w_norm * (1.0 + 3.0 * qq) * om * om * om;
      }
      double rho = d.cw_m * acc;
      double p = d.p0 * pow(rho / d.rho0, d.alpha) - d.beta;
      if (d.clamp && p < 0.0) p = 0.0;  // free-surface correction (Sec. 2.5)
      d.rho[i] = rho;
      d.p[i] = p;
    }
  });
}

// ---------------------------------------------------------------------------
// (a4) Shepard filter of the pressure and the FP32 pair records
// (v, c_C p~/d^2; spin, 1/d with d = rho/m_f).

static constexpr int CAP_SMOOTH = 1024;

template <bool GLOBAL>
__global__ __launch_bounds__(BS) void k_smooth_tiles(Dev d, int* ovf_list, int* ovf_cnt) {
  __shared__ TileHeader th;
  __shared__ double X[GLOBAL ? 1 : CAP_SMOOTH], Y[GLOBAL ? 1 : CAP_SMOOTH],
      Z[GLOBAL ? 1 : CAP_SMOOTH], PR[GLOBAL ? 1 : CAP_SMOOTH];
  for_bricks<GLOBAL>(d, th, CAP_SMOOTH, ovf_list, ovf_cnt, [&](const int* bc, int own_b,
                                                              int own_e) {
    const int tot = th.foff[FP];
    if (!GLOBAL && d.smooth) {
      for (int q = threadIdx.x; q < tot; q += BS) {
        int j = slot_to_index(th, q);
        D4 p = d.pos[j];
        X[q] = p.x;
        Y[q] = p.y;
        Z[q] = p.z;
        PR[q] = d.p[j];
      }
    }
    if (!GLOBAL) __syncthreads();
    const size_t np = (size_t)d.npad;
    const double inv_h = 1.0 / d.h;
    for (int i = own_b + threadIdx.x; i < own_e; i += BS) {
      const uint8_t ti = d.type[i];
      const double pi = d.p[i];
      double ps = pi;
      if (d.smooth && ti != T_OUTER) {
        const D4 xi = d.pos[i];
        double num = pi * d.W0, den = d.W0;
        const int cnt = d.nbr_cnt[i];
        for (int k = 0; k < cnt; ++k) {
          const int q = d.nbr16[(size_t)k * np + i];
          double xj, yj, zj, pj;
          if (GLOBAL) {
            int j = slot_to_index(th, q);
            D4 pp = d.pos[j];
            xj = pp.x;
            yj = pp.y;
            zj = pp.z;
            pj = d.p[j];
          } else {
            xj = X[q];
            yj = Y[q];
            zj = Z[q];
            pj = PR[q];
          }
          double ex = min_img(xi.x - xj, d.per[0], d.L[0], d.halfL[0]);
          double ey = min_img(xi.y - yj, d.per[1], d.L[1], d.halfL[1]);
          double ez = min_img(xi.z - zj, d.per[2], d.L[2], d.halfL[2]);
          double qq = sqrt(ex * ex + ey * ey + ez * ez) * inv_h;
          double om = fmax(1.0 - qq, 0.0);
          double w = d.w_norm * (1.0 + 3.0 * qq) * om * om * om;
          num += pj * w;
          den += w;
        }
        ps = num / den;
      }
      d.ps[i] = (float)ps;
      const double di = d.rho[i] / d.m_f;
      const D4 v = d.vel[i], w = d.om[i];
      F4 vr, wr;
      vr.x = (float)v.x;
      vr.y = (float)v.y;
      vr.z = (float)v.z;
      vr.w = (float)(d.coef_c * ps / (di * di));
      wr.x = (float)w.x;
      wr.y = (float)w.y;
      wr.z = (float)w.z;
      wr.w = (float)(1.0 / di);
      d.vrec[i] = vr;
      d.wrec[i] = wr;
    }
  });
}

// ---------------------------------------------------------------------------
// (a5) SDPD+a pair forces, Eqs. FijC, FijD, FijR, FijT, for fluid and
// inner-wall particles: FP32 math on FP64-differenced separations, FP32
// per-particle sums; outputs F^SDPD, its torque and the F^C + F^D sum.

template <bool NOISE, bool GLOBAL, int CAP>
__global__ __launch_bounds__(BS) void k_forces_tiles(Dev d, uint32_t step, int* ovf_list,
                                                    int* ovf_cnt) {
  constexpr int C = GLOBAL ? 1 : CAP;
  __shared__ TileHeader th;
  __shared__ double X[C], Y[C], Z[C];
  __shared__ F4 VR[C], WR[C];
  __shared__ uint32_t GID[(NOISE && !GLOBAL) ? CAP : 1];
  for_bricks<GLOBAL>(d, th, CAP, ovf_list, ovf_cnt, [&](const int* bc, int own_b, int own_e) {
    const int tot = th.foff[FP];
    if (!GLOBAL) {
      for (int q = threadIdx.x; q < tot; q += BS) {
        int j = slot_to_index(th, q);
        D4 p = d.pos[j];
        X[q] = p.x;
        Y[q] = p.y;
        Z[q] = p.z;
        VR[q] = d.vrec[j];
        WR[q] = d.wrec[j];
        if (NOISE) GID[q] = (uint32_t)d.gid[j];
      }
      __syncthreads();
    }
    const size_t np = (size_t)d.npad;
    for (int i = own_b + threadIdx.x; i < own_e; i += BS) {
      const uint8_t ti = d.type[i];
      float F0 = 0.f, F1 = 0.f, F2 = 0.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, N0 = 0.f, N1 = 0.f,
            N2 = 0.f;
      if (ti == T_FLUID || ti == T_INNER) {
        const D4 pi = d.pos[i];
        const F4 vi = d.vrec[i];
        const F4 wi = d.wrec[i];
        const uint32_t gi = NOISE ? (uint32_t)d.gid[i] : 0u;
        const int cnt = d.nbr_cnt[i];
        for (int k = 0; k < cnt; ++k) {
          const int q = d.nbr16[(size_t)k * np + i];
          double xj, yj, zj;
          F4 vj, wj;
          uint32_t gj = 0;
          if (GLOBAL) {
            int j = slot_to_index(th, q);
            D4 pj = d.pos[j];
            xj = pj.x;
            yj = pj.y;
            zj = pj.z;
            vj = d.vrec[j];
            wj = d.wrec[j];
            if (NOISE) gj = (uint32_t)d.gid[j];
          } else {
            xj = X[q];
            yj = Y[q];
            zj = Z[q];
            vj = VR[q];
            wj = WR[q];
            if (NOISE) gj = GID[q];
          }
          const double dx_ = min_img(pi.x - xj, d.per[0], d.L[0], d.halfL[0]);
          const double dy_ = min_img(pi.y - yj, d.per[1], d.L[1], d.halfL[1]);
          const double dz_ = min_img(pi.z - zj, d.per[2], d.L[2], d.halfL[2]);
          const double r2d = dx_ * dx_ + dy_ * dy_ + dz_ * dz_;
          const float rx = (float)dx_, ry = (float)dy_, rz = (float)dz_;
          const float inv_r = __builtin_amdgcn_rsqf((float)r2d);
          const float r = (float)r2d * inv_r;
          const float ex = rx * inv_r, ey = ry * inv_r, ez = rz * inv_r;
          // 1 - r/h = (h^2 - r^2) / (h (h + r)), the difference taken in FP64
          // so that pairs close to the cut-off keep full FP32 relative precision
          const float omq =
              fmaxf((float)(d.h2 - r2d) * d.inv_hf * __builtin_amdgcn_rcpf(d.hf + r), 0.0f);
          const float Fk = d.cFf * omq * omq;  // F(r) = -W'(r)/r, Eq. F
          // Pair force = along-e part + transverse part.  The torque takes the
          // transverse part only (e x e = 0), which keeps the FP32 cross
          // product free of the cancellation of the dominant pressure term.
          // conservative force, Eq. FijC: (p_i/d_i^2 + p_j/d_j^2) F r_ij
          const float pc = (vi.w + vj.w) * Fk;
          // F / (d_i d_j): the two inverse densities multiply symmetrically
          // so that F_ji = -F_ij holds bit for bit
          const float fdd = Fk * (wi.w * wj.w);
          // dissipative force, Eq. FijD: -ga v_ij - (ga + 2 gb)/3 (e.v_ij) e
          const float vx = vi.x - vj.x, vy = vi.y - vj.y, vz = vi.z - vj.z;
          const float ev = ex * vx + ey * vy + ez * vz;
          const float cde = d.kBf * fdd * ev;
          const float cdv = d.kAf * fdd;
          float tx = cdv * vx, ty = cdv * vy, tz = cdv * vz;
          const float cx_ = pc * rx + cde * ex + tx;
          const float cy_ = pc * ry + cde * ey + ty;
          const float cz_ = pc * rz + cde * ez + tz;
          C0 += cx_;
          C1 += cy_;
          C2 += cz_;
          // rotational force, Eq. FijR: -gamma^a (r_ij / 2) x (w_i + w_j)
          const float sx = wi.x + wj.x, sy = wi.y + wj.y, sz = wi.z + wj.z;
          const float gr = d.kRf * fdd;
          const float rrx = gr * (ry * sz - rz * sy);
          const float rry = gr * (rz * sx - rx * sz);
          const float rrz = gr * (rx * sy - ry * sx);
          float fx = cx_ + rrx, fy = cy_ + rry, fz = cz_ + rrz;
          tx += rrx;
          ty += rry;
          tz += rrz;
          if (NOISE) {
            // thermal force, Eq. FijT with dW^S = sym(dW) - tr(dW)/3
            float z[9];
            pair_normals(gi, gj, step, d.key0, d.key1, z);
            const float sa = 2.0f * sqrtf(d.kTf * d.CAf * fdd);
            const float sb = 2.0f * sqrtf(d.kTf * d.CBf * fdd);
            const float tr3 = (z[0] + z[4] + z[8]) * (1.0f / 3.0f);
            const float s01 = 0.5f * (z[1] + z[3]), s02 = 0.5f * (z[2] + z[6]),
                        s12 = 0.5f * (z[5] + z[7]);
            const float se0 = (z[0] - tr3) * ex + s01 * ey + s02 * ez;
            const float se1 = s01 * ex + (z[4] - tr3) * ey + s12 * ez;
            const float se2 = s02 * ex + s12 * ey + (z[8] - tr3) * ez;
            const float ca = d.cT * d.inv_sqrt_dtf * sa;
            const float cb = d.cT * d.inv_sqrt_dtf * sb * tr3;
            fx += ca * se0 + cb * ex;
            fy += ca * se1 + cb * ey;
            fz += ca * se2 + cb * ez;
            tx += ca * se0;
            ty += ca * se1;
            tz += ca * se2;
          }
          F0 += fx;
          F1 += fy;
          F2 += fz;
          // torque: lever dx/2 along -e_ij (Sec. 2.6), lever applied below
          N0 += ey * tz - ez * ty;
          N1 += ez * tx - ex * tz;
          N2 += ex * ty - ey * tx;
        }
        N0 *= -d.leverf;
        N1 *= -d.leverf;
        N2 *= -d.leverf;
      }
      float* o = d.fout;
      o[0 * np + i] = F0;
      o[1 * np + i] = F1;
      o[2 * np + i] = F2;
      o[3 * np + i] = N0;
      o[4 * np + i] = N1;
      o[5 * np + i] = N2;
      o[6 * np + i] = C0;
      o[7 * np + i] = C1;
      o[8 * np + i] = C2;
    }
  });
}

// ---------------------------------------------------------------------------
// launchers: the LDS pass over all bricks, then the global pass over the
// bricks it deferred (a launch that exits at once when there are none)

void launch_build_density(const Dev& d, hipStream_t st) {
  launch_fill_i32(d.ovf_cnt + 0, 0, 1, st);
  k_build_tiles<false><<<brick_blocks(d.g.nbricks), BS, 0, st>>>(d, d.ovf_list, d.ovf_cnt + 0);
  k_build_tiles<true><<<OVF_BLOCKS, BS, 0, st>>>(d, d.ovf_list, d.ovf_cnt + 0);
}

void launch_smooth(const Dev& d, hipStream_t st) {
  int* list = d.ovf_list + d.g.nbricks;
  launch_fill_i32(d.ovf_cnt + 1, 0, 1, st);
  k_smooth_tiles<false><<<brick_blocks(d.g.nbricks), BS, 0, st>>>(d, list, d.ovf_cnt + 1);
  k_smooth_tiles<true><<<OVF_BLOCKS, BS, 0, st>>>(d, list, d.ovf_cnt + 1);
}

void launch_fluid_forces(const Dev& d, uint32_t step, bool noise, hipStream_t st) {
  const int nb = brick_blocks(d.g.nbricks);
  int* list = d.ovf_list + 2 * (size_t)d.g.nbricks;
  launch_fill_i32(d.ovf_cnt + 2, 0, 1, st);
  if (noise) {
    k_forces_tiles<true, false, 832><<<nb, BS, 0, st>>>(d, step, list, d.ovf_cnt + 2);
    k_forces_tiles<true, true, 832><<<OVF_BLOCKS, BS, 0, st>>>(d, step, list, d.ovf_cnt + 2);
  } else {
    k_forces_tiles<false, false, 896><<<nb, BS, 0, st>>>(d, step, list, d.ovf_cnt + 2);
    k_forces_tiles<false, true, 896><<<OVF_BLOCKS, BS, 0, st>>>(d, step, list, d.ovf_cnt + 2);
  }
}

// ---------------------------------------------------------------------------
// neighbour columns k0..k0+kn-1 of every particle as ids (-1 past a row's
// end), for the export of the neighbour sets

__global__ __launch_bounds__(BS) void k_nbr_cols_tiles(Dev d, int k0, int kn, int* out) {
  __shared__ TileHeader th;
  const int rank = blockIdx.x;
  if (rank >= d.g.nbricks) return;
  if (d.cstart[rank * 64] == d.cstart[rank * 64 + 64]) return;
  int bc[3], own_b, own_e;
  tile_setup(d, rank, th, bc, own_b, own_e);
  const size_t np = (size_t)d.npad;
  for (int i = own_b + threadIdx.x; i < own_e; i += BS) {
    const int cnt = d.nbr_cnt[i];
    for (int k = 0; k < kn; ++k) {
      int kk = k0 + k;
      out[(size_t)k * np + i] =
          kk < cnt ? d.gid[slot_to_index(th, d.nbr16[(size_t)kk * np + i])] : -1;
    }
  }
}

void launch_nbr_cols(const Dev& d, int k0, int kn, int* out, hipStream_t st) {
  k_nbr_cols_tiles<<<brick_blocks(d.g.nbricks), BS, 0, st>>>(d, k0, kn, out);
}

}  // namespace sdpdem
