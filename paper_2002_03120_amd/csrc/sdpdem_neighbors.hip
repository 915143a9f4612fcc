// sdpdem_neighbors.hip -- neighbour build with density, pressure filter and
// SDPD pair forces: one thread per particle in cell-sorted order, blocks
// mapped to XCDs in contiguous chunks, neighbour data gathered through L1/L2
// (the sorted order keeps a wave's neighbourhood compact).
#include <hip/hip_ext.h>

#include "sdpdem_device.h"

namespace sdpdem {

// ---------------------------------------------------------------------------
// (a2)+(a3) neighbour sets {j : r_ij^2 < h^2} (double precision, no
// contraction) fused with the density summation (Eq. compdens), the
// equation of state (Eq. prtcpres) and the free-surface clamp.  The
// stencil is walked row by row; the cells of a row are one contiguous slice
// of the sorted arrays unless the row wraps.  With CAND (candidate reuse)
// the walk reaches h + skin and also keeps every partner within it, with
// the positions it saw, for the list builds until the next search.

// density and pressure of particle i from its kernel sum, and its
// (position, pressure) record for the filter
__device__ __forceinline__ void finish_density(const Dev& d, int i, const D4& pi, double acc) {
  const double rho = d.cw_m * acc;
  double p = d.p0 * pow(rho / d.rho0, d.alpha) - d.beta;
  if (d.clamp && p < 0.0) p = 0.0;  // free-surface correction (Sec. 2.5)
  d.rho[i] = rho;
  d.p[i] = p;
  d.xp[i] = D4{pi.x, pi.y, pi.z, p};
}

__device__ __forceinline__ void outer_wall_fields(const Dev& d, int i, const D4& pi) {
  d.nbr_cnt[i] = 0;
  d.rho[i] = d.rho0;
  d.p[i] = d.p_ref;
  d.xp[i] = D4{pi.x, pi.y, pi.z, d.p_ref};
}

// after_drift: the build between the two passes of a step, at the
// positions the step's drift made; otherwise a build ahead of the first
// pass, at the positions the previous step's drift made
template <bool CAND>
__device__ __forceinline__ void build_density(const Dev& d, int after_drift) {
  // a search resets the moved flag: positions are measured from here on
  if (CAND && blockIdx.x == 0 && threadIdx.x == 0) {
    d.moved[0] = 0;
    d.sstep[0] = d.dstep[0] - (after_drift ? 0 : 1);
  }
  int i;
  const int b = blk_box(d, i);
  if (b < 0) return;
  const BoxD& B = d.boxes[b];
  if (i >= B.first + B.count) return;
  uint8_t ti = d.type[i];
  const D4 pi = d.pos[i];
  if (CAND) d.xref[i] = pi;
  if (ti == T_OUTER) {
    outer_wall_fields(d, i, pi);
    if (CAND) d.cand_cnt[i] = 0;
    return;
  }
  const Geo G = geo_of(B);
  const Grid gr = B.g;
  const int coff = B.cell_off;
  int oob = 0;
  const int cc[3] = {cell_coord(pi.x, gr, 0, &oob), cell_coord(pi.y, gr, 1, &oob),
                     cell_coord(pi.z, gr, 2, &oob)};
  const double h2 = d.h2, inv_h = d.inv_h;
  const double R = CAND ? d.hc : d.h;
  const double R2 = CAND ? d.hc2 : h2;
  double acc = d.W0;
  int cnt = 0, ccnt = 0;
  const size_t npad = (size_t)d.npad;
  int* const nb = d.nbr + i;
  int* const cb = CAND ? d.cand + i : nullptr;
  auto cells = [&](int k0, int k1) {
    const int jb = d.cstart[k0];
    const int je = d.cstart[k1];
    for (int j = jb; j < je; ++j) {
      const D4 pj = d.pos[j];
      double ex = pi.x - pj.x, ey = pi.y - pj.y, ez = pi.z - pj.z;
      min_img_fast(G, ex, ey, ez);
      const double r2 = r2_exact(ex, ey, ez);
      if (r2 < R2 && j != i) {
        if (CAND) {
          if (ccnt < d.maxcand) cb[(size_t)ccnt * npad] = j;
          ++ccnt;
        }
        if (!CAND || r2 < h2) {
          const double q = sqrt_nr(r2) * inv_h;
          const double om = 1.0 - q;
          if (cnt < d.maxn) nb[(size_t)cnt * npad] = j;
          ++cnt;
          acc += d.w_norm * (1.0 + 3.0 * q) * om * om * om;
        }
      }
    }
  };
  // a run of cells, then the outer walls binned in the same cells
  const int woff = B.wall_off;
  auto run = [&](int k0, int k1) {
    cells(k0, k1);
    if (woff) cells(k0 + woff, k1 + woff);
  };
  // cells of R or more: the whole 27-cell stencil (lanes of a cell walk the
  // same runs in step); smaller cells: the rows and x cells within R only
  const int kr = reach_cells(gr, R);
  if (kr == 1)
    for_stencil<false>(G, gr, coff, pi.x, pi.y, pi.z, R, cc, 1, run);
  else
    for_stencil_pruned(G, gr, coff, pi.x, pi.y, pi.z, R, cc, kr, run);
  if (cnt > d.maxn || (CAND && ccnt > d.maxcand)) {
    atomicOr(d.status, ST_NBR_OVERFLOW);
    cnt = min(cnt, d.maxn);
    ccnt = min(ccnt, d.maxcand);
  }
  d.nbr_cnt[i] = cnt;
  if (CAND) d.cand_cnt[i] = ccnt;
  finish_density(d, i, pi, acc);
}

// eight waves per SIMD for the plain search; the candidate search holds
// more state and spills below 96 registers, so it takes five
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(8))) void k_build_density(Dev d) {
  build_density<false>(d, 0);
}
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(5))) void k_build_candidates(Dev d, int after_drift) {
  build_density<true>(d, after_drift);
}

void launch_build_density(const Dev& d, bool cand, bool after_drift, hipStream_t st) {
  if (cand)
    k_build_candidates<<<d.nblk, BS, 0, st>>>(d, after_drift ? 1 : 0);
  else
    k_build_density<<<d.nblk, BS, 0, st>>>(d);
}

// The lists of a drift that kept every particle within skin/2 of where the
// last search saw it: a partner within h now was within h + skin then, so
// the exact test over the candidates (in the same FP64 arithmetic) gives
// the same set as a search.  Density, pressure and the filter's record as
// in the search.
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(8))) void k_filter_density(Dev d) {
  int i;
  const int b = blk_box<true>(d, i);
  if (b < 0) return;
  const BoxD& B = d.boxes[b];
  if (i >= B.first + B.count) return;
  const uint8_t ti = d.type[i];
  const D4 pi = d.pos[i];
  if (ti == T_OUTER) {
    outer_wall_fields(d, i, pi);
    return;
  }
  const Geo G = geo_of(B);
  const double h2 = d.h2, inv_h = d.inv_h;
  double acc = d.W0;
  int cnt = 0;
  const size_t npad = (size_t)d.npad;
  int* const nb = d.nbr + i;
  const int* const cb = d.cand + i;
  const int cc = d.cand_cnt[i];
  // software pipeline: the position of candidate k+1 and the index of
  // candidate k+2 are in flight while candidate k is tested (past the end
  // the loads fetch the particle's own, unused, entries)
  int jn = cc > 0 ? cb[0] : i;
  D4 pn = d.pos[jn];
  int jnn = cc > 1 ? cb[npad] : i;
  for (int k = 0; k < cc; ++k) {
    const int j = jn;
    const D4 pj = pn;
    jn = jnn;
    pn = d.pos[jn];
    jnn = k + 2 < cc ? cb[(size_t)(k + 2) * npad] : i;
    double ex = pi.x - pj.x, ey = pi.y - pj.y, ez = pi.z - pj.z;
    min_img_fast(G, ex, ey, ez);
    const double r2 = r2_exact(ex, ey, ez);
    if (r2 < h2) {
      const double q = sqrt_nr(r2) * inv_h;
      const double om = 1.0 - q;
      if (cnt < d.maxn) nb[(size_t)cnt * npad] = j;
      ++cnt;
      acc += d.w_norm * (1.0 + 3.0 * q) * om * om * om;
    }
  }
  if (cnt > d.maxn) {
    atomicOr(d.status, ST_NBR_OVERFLOW);
    cnt = d.maxn;
  }
  d.nbr_cnt[i] = cnt;
  finish_density(d, i, pi, acc);
}

void launch_filter_density(const Dev& d, hipStream_t st) {
  k_filter_density<<<d.nablk, BS, 0, st>>>(d);
}

// ---------------------------------------------------------------------------
// (a4) Shepard filter of the pressure (weights recomputed from the FP64
// positions) and the pair records of the force pass.

template <bool ACT>
__global__ __launch_bounds__(BS) void k_smooth(Dev d) {
  int i;
  const int b = blk_box<ACT>(d, i);
  if (b < 0) return;
  const BoxD& B = d.boxes[b];
  if (i >= B.first + B.count) return;
  const uint8_t ti = d.type[i];
  const D4 x = d.xp[i];  // position and pressure
  const double pi = x.w;
  const Geo G = geo_of(B);
  double ps = pi;
  if (d.smooth && ti != T_OUTER) {
    double num = pi * d.W0, den = d.W0;
    const int cnt = d.nbr_cnt[i];
    const size_t npad = (size_t)d.npad;
    const int* nb = d.nbr + i;
    const double inv_h = d.inv_h;
    for (int k = 0; k < cnt; ++k) {
      const int j = nb[(size_t)k * npad];
      const D4 xj = d.xp[j];  // one 32-byte record: position and pressure
      double ex = x.x - xj.x, ey = x.y - xj.y, ez = x.z - xj.z;
      min_img_fast(G, ex, ey, ez);
      const double q = sqrt_nr(r2_exact(ex, ey, ez)) * inv_h;
      const double om = fmax(1.0 - q, 0.0);
      const double w = d.w_norm * (1.0 + 3.0 * q) * om * om * om;
      num += xj.w * w;
      den += w;
    }
    ps = num / den;
  }
  d.ps[i] = (float)ps;
  const double di = d.rho[i] / d.m_f;
  const D4 v = d.vel[i], w = d.om[i];
  PR r;
  r.x = x.x;
  r.y = x.y;
  r.z = x.z;
  r.vx = (float)v.x;
  r.vy = (float)v.y;
  r.vz = (float)v.z;
  r.pc = (float)(d.coef_c * ps / (di * di));
  r.wx = (float)w.x;
  r.wy = (float)w.y;
  r.wz = (float)w.z;
  r.invd = (float)(1.0 / di);
  r.gid = d.gid[i];
  r.type = ti;
  d.prec[i] = r;
}

// after a search over every particle (the outer walls' records too: the
// sort may have moved them), after a candidate filter over the active parts
void launch_smooth(const Dev& d, bool all, hipStream_t st) {
  if (all)
    k_smooth<false><<<d.nblk, BS, 0, st>>>(d);
  else
    k_smooth<true><<<d.nablk, BS, 0, st>>>(d);
}

// ---------------------------------------------------------------------------
// (a5) SDPD+a pair forces, Eqs. FijC, FijD, FijR, FijT, for fluid and
// inner-wall particles: FP32 math on FP64-differenced separations, FP32
// per-particle sums; outputs F^SDPD, its torque and the F^C + F^D sum.

template <bool NOISE, bool STRESS>
__global__ __launch_bounds__(BS) void k_fluid_forces(Dev d) {
  int i;
  const int b = blk_box<true>(d, i);
  if (b < 0) return;
  const BoxD& B = d.boxes[b];
  if (i >= B.first + B.count) return;
  const uint8_t ti = d.type[i];
  float F0 = 0.f, F1 = 0.f, F2 = 0.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, N0 = 0.f, N1 = 0.f, N2 = 0.f;
  float Wzx = 0.f;
  if (ti == T_FLUID || ti == T_INNER) {
    const PR ri = load_pr(d.prec, i);
    const uint32_t ib = B.id_base;
    const uint32_t gi = (uint32_t)ri.gid - ib;  // box-local noise index
    const int cnt = d.nbr_cnt[i];
    const int* nb = d.nbr + i;
    const size_t npad = (size_t)d.npad;
    const Geo G = geo_of(B);
    const bool le = G.le;
    const float jump = (float)G.le_jump;
    const bool noise = NOISE && B.noise;
    const float kT = B.kTf;
    const uint32_t key0 = B.key0, key1 = B.key1;
    const uint32_t step = NOISE ? (uint32_t)d.dstep[0] : 0u;  // noise counter
    // the index of slot k+1 is in flight while slot k is evaluated (holding
    // the next record too costs 19 registers: 7 waves per SIMD instead of 8,
    // and the kernel is 4 % slower)
    int jn = cnt > 0 ? nb[0] : i;
    for (int k = 0; k < cnt; ++k) {
      const PR rj = load_pr(d.prec, jn);
      jn = k + 1 < cnt ? nb[(size_t)(k + 1) * npad] : i;
      double dx_ = ri.x - rj.x, dy_ = ri.y - rj.y, dz_ = ri.z - rj.z;
      const int kz = NOISE ? min_img_fast(G, dx_, dy_, dz_) : min_img_box(G, dx_, dy_, dz_);
      const double r2d = dx_ * dx_ + dy_ * dy_ + dz_ * dz_;
      const float rx = (float)dx_, ry = (float)dy_, rz = (float)dz_;
      const float inv_r = __builtin_amdgcn_rsqf((float)r2d);
      const float r = (float)r2d * inv_r;
      const float ex = rx * inv_r, ey = ry * inv_r, ez = rz * inv_r;
      // 1 - r/h = (h^2 - r^2) / (h (h + r)), the difference taken in FP64 so
      // that pairs close to the cut-off keep full FP32 relative precision
      const float omq =
          fmaxf((float)(d.h2 - r2d) * d.inv_hf * __builtin_amdgcn_rcpf(d.hf + r), 0.0f);
      const float Fk = d.cFf * omq * omq;  // F(r) = -W'(r)/r, Eq. F
      // Pair force = along-e part + transverse part.  The torque takes the
      // transverse part only (e x e = 0), which keeps the FP32 cross product
      // free of the cancellation of the dominant pressure term.
      // conservative force, Eq. FijC: (p_i/d_i^2 + p_j/d_j^2) F r_ij
      const float pc = (ri.pc + rj.pc) * Fk;
      // F / (d_i d_j): the two inverse densities multiply symmetrically so
      // that F_ji = -F_ij holds bit for bit
      const float fdd = Fk * (ri.invd * rj.invd);
      // dissipative force, Eq. FijD: -ga v_ij - (ga + 2 gb)/3 (e.v_ij) e; a
      // partner seen through a sheared z face moves with its image velocity
      float vx = ri.vx - rj.vx;
      if (le) vx = vx - (float)kz * jump;
      const float vy = ri.vy - rj.vy, vz = ri.vz - rj.vz;
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
      const float sx = ri.wx + rj.wx, sy = ri.wy + rj.wy, sz = ri.wz + rj.wz;
      const float gr = d.kRf * fdd;
      const float rrx = gr * (ry * sz - rz * sy);
      const float rry = gr * (rz * sx - rx * sz);
      const float rrz = gr * (rx * sy - ry * sx);
      float fx = cx_ + rrx, fy = cy_ + rry, fz = cz_ + rrz;
      tx += rrx;
      ty += rry;
      tz += rrz;
      if (noise) {
        // thermal force, Eq. FijT: (sa dW^S + sb tr(dW)/3 1) e for a matrix
        // of independent increments is Gaussian with variance 1/2 across e
        // and sa^2 2/3 + sb^2 1/3 along it (in units of sa^2 and dt), the
        // two parts independent: s_ij P_perp z / sqrt 2 with z = (z0, z1,
        // z2) plus z3 along e, s_ij = +1 for gid_i < gid_j (F_ji = -F_ij)
        float z[4];
        const uint32_t gj = (uint32_t)rj.gid - ib;
        pair_normals(gi, gj, step, key0, key1, z);
        const float sa2 = 4.0f * kT * d.CAf * fdd, sb2 = 4.0f * kT * d.CBf * fdd;
        const float ze = z[0] * ex + z[1] * ey + z[2] * ez;
        const float px = z[0] - ze * ex, py = z[1] - ze * ey, pz = z[2] - ze * ez;
        const float cn = d.cT * d.inv_sqrt_dtf;
        const float cp = cn * sqrtf(sa2) * (gi < gj ? 0.70710678118654752f : -0.70710678118654752f);
        const float cq = cn * sqrtf(sa2 * (2.0f / 3.0f) + sb2 * (1.0f / 3.0f)) * z[3];
        fx += cp * px + cq * ex;
        fy += cp * py + cq * ey;
        fz += cp * pz + cq * ez;
        // the torque takes the part across e (e x e = 0)
        tx += cp * px;
        ty += cp * py;
        tz += cp * pz;
      }
      F0 += fx;
      F1 += fy;
      F2 += fz;
      // torque: lever dx/2 along -e_ij (Sec. 2.6), lever applied below
      N0 += ey * tz - ez * ty;
      N1 += ez * tx - ex * tz;
      N2 += ex * ty - ey * tx;
      if (STRESS) {
        // virial r_z F_x: half of a pair that j evaluates too, all of a
        // pair with a rigid or outer-wall partner (it does not)
        const float c = (rj.type == T_FLUID || rj.type == T_INNER) ? 0.5f : 1.0f;
        Wzx += c * rz * fx;
      }
    }
    N0 *= -d.leverf;
    N1 *= -d.leverf;
    N2 *= -d.leverf;
  }
  const size_t np = (size_t)d.npad;
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
  if (STRESS) o[12 * np + i] = Wzx;
}

void launch_fluid_forces(const Dev& d, bool noise, hipStream_t st, hipEvent_t t0,
                         hipEvent_t t1) {
  auto k = noise ? (d.stress ? k_fluid_forces<true, true> : k_fluid_forces<true, false>)
                 : (d.stress ? k_fluid_forces<false, true> : k_fluid_forces<false, false>);
  if (t0 && t1) {
    // the dispatch itself stamps the two events (no marker packets around
    // the kernel, which would stall the stream)
    Dev arg = d;
    void* args[] = {&arg};
    if (hipExtLaunchKernel(reinterpret_cast<const void*>(k), dim3(d.nablk), dim3(BS), args, 0, st,
                           t0, t1, 0) == hipSuccess)
      return;
  }
  k<<<d.nablk, BS, 0, st>>>(d);
}

// neighbour columns k0..k0+kn-1 as ids (-1 past a row's end), for export
__global__ __launch_bounds__(BS) void k_nbr_cols(Dev d, int k0, int kn, int* out) {
  const int i = xcd_tid();
  if (i >= d.n) return;
  const int cnt = d.nbr_cnt[i];
  const size_t np = (size_t)d.npad;
  for (int k = 0; k < kn; ++k) {
    const int kk = k0 + k;
    out[(size_t)k * np + i] = kk < cnt ? d.gid[d.nbr[(size_t)kk * np + i]] : -1;
  }
}

void launch_nbr_cols(const Dev& d, int k0, int kn, int* out, hipStream_t st) {
  k_nbr_cols<<<nblocks(d.n), BS, 0, st>>>(d, k0, kn, out);
}

}  // namespace sdpdem
