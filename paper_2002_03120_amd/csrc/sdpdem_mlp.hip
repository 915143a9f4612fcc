// sdpdem_mlp.hip -- the viscosity surrogate: a 4-64-64-64-1 SiLU MLP with
// bfloat16 parameters, float32 activations and float32 accumulation on the
// matrix cores, trained with Adam.  Inference runs the hidden layers on the
// bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16, activations split into
// three exact bfloat16 parts); a training step (forward, MSE loss,
// backward, Adam) is one workgroup on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32), so every reduction has a fixed order and a
// step is bit-for-bit repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "sdpdem.h"
#include "sdpdem_mlp.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int NP = SDPDEM_MLP_PARAMS;
constexpr int HID = 64;
constexpr int MAXB = SDPDEM_MLP_MAX_BATCH;
// parameter offsets: W1 [4 x 64], b1, W2 [64 x 64], b2, W3 [64 x 64], b3, W4 [64], b4
constexpr int OW1 = 0, OB1 = 256, OW2 = 320, OB2 = 4416, OW3 = 4480, OB3 = 8576, OW4 = 8640,
              OB4 = 8704;
constexpr int OW[3] = {OW1, OW2, OW3};
constexpr int OB[3] = {OB1, OB2, OB3};
static_assert(OB4 + 1 == NP, "parameter layout");

struct Norm {
  float mean[4], inv_std[4];
};

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// round to nearest, ties to even
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// logistic function from the hardware exp2 and reciprocal (about one ulp
// each; the FP64 oracle agrees to the tolerance of the parity tests)
__device__ __forceinline__ float sigm(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.44269504088896341f * z));
}
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

// acc += A[16 x K] B[K x 16] on the matrix cores, K a multiple of 4.  Lane
// (r = lane % 16, q = lane / 16) supplies A(r, k0 + q) and B(k0 + q, r) per
// step; on return it holds C(4q + v, r) in acc[v].
template <class FA, class FB>
__device__ __forceinline__ v4f mfma_tile(int K, FA fa, FB fb, v4f acc) {
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += 4)
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fa(r, k0 + q), fb(k0 + q, r), acc, 0, 0, 0);
  return acc;
}

// ---------------------------------------------------------------------------
// inference on the bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16).  The
// parameters are bfloat16 values already; an FP32 activation is the exact
// sum of three bfloat16 parts (its top 8 significant bits, the next 8, the
// last 8), so three bf16 products accumulated in FP32 give the FP32
// product, and the layer equals its FP32 evaluation up to the order of the
// sums.  A block stages the hidden layers' weights, transposed, in LDS once
// and its wavefronts then take groups of 16 rows in turn; each wavefront
// keeps its 16 x 64 activation tiles in LDS.

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8u16 __attribute__((ext_vector_type(8)));

constexpr int LDA = HID + 4;  // padded row stride of the activation tiles
constexpr int PRED_WAVES = 4;

// x = hi + mid + lo exactly, each part a bfloat16 (truncations of x and of
// the remainders: every part holds at most 8 significant bits)
__device__ __forceinline__ void split3(float x, unsigned short& h, unsigned short& m,
                                       unsigned short& l) {
  const uint32_t uh = __float_as_uint(x) & 0xFFFF0000u;
  const float r1 = x - __uint_as_float(uh);
  const uint32_t um = __float_as_uint(r1) & 0xFFFF0000u;
  const float r2 = r1 - __uint_as_float(um);
  h = (unsigned short)(uh >> 16);
  m = (unsigned short)(um >> 16);
  l = (unsigned short)(__float_as_uint(r2) >> 16);
}

__global__ __launch_bounds__(64 * PRED_WAVES) void k_mlp_predict(const uint16_t* __restrict__ wq,
                                                                 Norm nrm,
                                                                 const float* __restrict__ x,
                                                                 float* __restrict__ y, int64_t n,
                                                                 int64_t groups_per_wave) {
  // W2^T and W3^T: wt[l][j * HID + k] = W_{l+2}[k][j] (bf16 bits)
  __shared__ __attribute__((aligned(16))) unsigned short wt[2][HID * HID];
  __shared__ float w1[4 * HID], bias[3][HID], w4[HID + 1];
  __shared__ float act[PRED_WAVES][2][16 * LDA];
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * HID * HID; e += 64 * PRED_WAVES) {
    const int l = e / (HID * HID), rem = e % (HID * HID), k = rem / HID, j = rem % HID;
    wt[l][j * HID + k] = wq[OW[l + 1] + k * HID + j];
  }
  for (int e = tid; e < 4 * HID; e += 64 * PRED_WAVES) w1[e] = bf16_to_f32(wq[OW1 + e]);
  for (int e = tid; e < 3 * HID; e += 64 * PRED_WAVES)
    bias[e / HID][e % HID] = bf16_to_f32(wq[OB[e / HID] + e % HID]);
  for (int e = tid; e <= HID; e += 64 * PRED_WAVES) w4[e] = bf16_to_f32(wq[OW4 + e]);
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63, r = lane & 15, q = lane >> 4;
  float* h0 = act[w][0];
  float* h1 = act[w][1];
  const int64_t wave = (int64_t)blockIdx.x * PRED_WAVES + w;
  const int64_t nwaves = (int64_t)gridDim.x * PRED_WAVES;
  for (int64_t it = 0; it < groups_per_wave; ++it) {
    const int64_t row0 = (wave + it * nwaves) * 16;
    if (row0 >= n) break;  // a wavefront's own loop: no block barrier inside
    // layer 1: K = 4 features, one FP32 MFMA per 16 x 16 tile
    {
      const int64_t row = row0 + r;
      const float a = row < n ? (x[row * 4 + q] - nrm.mean[q]) * nrm.inv_std[q] : 0.0f;
      for (int jt = 0; jt < 4; ++jt) {
        const float b0 = bias[0][16 * jt + r];
        v4f acc = {b0, b0, b0, b0};
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, w1[q * HID + 16 * jt + r], acc, 0, 0, 0);
        for (int v = 0; v < 4; ++v) h0[(4 * q + v) * LDA + 16 * jt + r] = silu(acc[v]);
      }
    }
    // layers 2 and 3: K = 64 as two chunks of 32; lane (r, q) supplies
    // A(r, 32c + 8q .. + 7) and B(32c + 8q .. + 7, r), holds C(4q + v, r)
    for (int l = 0; l < 2; ++l) {
      const float* hin = l == 0 ? h0 : h1;
      float* hout = l == 0 ? h1 : h0;
      v8u16 ah[2], am[2], al[2];
      for (int c = 0; c < 2; ++c)
        for (int e = 0; e < 8; ++e) {
          unsigned short hh, mm, ll;
          split3(hin[r * LDA + 32 * c + 8 * q + e], hh, mm, ll);
          ah[c][e] = hh;
          am[c][e] = mm;
          al[c][e] = ll;
        }
      for (int jt = 0; jt < 4; ++jt) {
        const float bj = bias[l + 1][16 * jt + r];
        v4f acc = {bj, bj, bj, bj};
        for (int c = 0; c < 2; ++c) {
          const v8u16 bw =
              *reinterpret_cast<const v8u16*>(&wt[l][(16 * jt + r) * HID + 32 * c + 8 * q]);
          const v8bf b = __builtin_bit_cast(v8bf, bw);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, ah[c]), b, acc,
                                                        0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, am[c]), b, acc,
                                                        0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, al[c]), b, acc,
                                                        0, 0, 0);
        }
        for (int v = 0; v < 4; ++v) hout[(4 * q + v) * LDA + 16 * jt + r] = silu(acc[v]);
      }
    }
    // output layer: lanes (r, q) sum k in [16q, 16q + 16), then across q
    float p = 0.0f;
    for (int k = 16 * q; k < 16 * q + 16; ++k) p += h0[r * LDA + k] * w4[k];
    p += __shfl_xor(p, 16, 64);
    p += __shfl_xor(p, 32, 64);
    const int64_t row = row0 + r;
    if (q == 0 && row < n) y[row] = p + w4[HID];
  }
}

// ---------------------------------------------------------------------------
// training step: one workgroup of 4 wavefronts

struct Train {
  float* master;
  float* m;
  float* v;
  float* grad;
  uint16_t* wq;
  float* loss;
  float* xn;   // [MAXB x 4]
  float* z;    // [3][MAXB x 64]
  float* h;    // [3][MAXB x 64]
  float* dz0;  // [MAXB x 64]
  float* dz1;  // [MAXB x 64]
  float* dy;   // [MAXB]
};

__global__ __launch_bounds__(256) void k_mlp_train(Train T, Norm nrm, const float* __restrict__ x,
                                                   const float* __restrict__ t, int B, int update,
                                                   float lr, float b1, float b2, float eps,
                                                   float bc1, float bc2) {
  __shared__ float red[256];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r = lane & 15, q = lane >> 4;
  const int Bp = (B + 15) & ~15;
  const int ngroups = Bp / 16;
  // inputs, normalised; padding rows are zero
  for (int k = tid; k < Bp * 4; k += 256) {
    const int i = k >> 2, f = k & 3;
    T.xn[k] = i < B ? (x[k] - nrm.mean[f]) * nrm.inv_std[f] : 0.0f;
  }
  __syncthreads();
  // forward: z_l = h_{l-1} W_l + b_l, h_l = silu(z_l)
  for (int l = 0; l < 3; ++l) {
    const int K = l == 0 ? 4 : HID;
    const float* hin = l == 0 ? T.xn : T.h + (size_t)(l - 1) * MAXB * HID;
    float* zl = T.z + (size_t)l * MAXB * HID;
    float* hl = T.h + (size_t)l * MAXB * HID;
    for (int item = w; item < ngroups * 4; item += 4) {
      const int g = item >> 2, jt = item & 3;
      const float bias = bf16_to_f32(T.wq[OB[l] + 16 * jt + r]);
      v4f acc = {bias, bias, bias, bias};
      acc = mfma_tile(
          K, [&](int i, int k) { return hin[(16 * g + i) * K + k]; },
          [&](int k, int j) { return bf16_to_f32(T.wq[OW[l] + k * HID + 16 * jt + j]); }, acc);
      for (int v = 0; v < 4; ++v) {
        const int idx = (16 * g + 4 * q + v) * HID + 16 * jt + r;
        zl[idx] = acc[v];
        hl[idx] = silu(acc[v]);
      }
    }
    __syncthreads();
  }
  // output, residual, dL/dy = 2 (y - t) / B and the loss
  const float* h3 = T.h + (size_t)2 * MAXB * HID;
  float part = 0.0f;
  for (int i = tid; i < Bp; i += 256) {
    float y = bf16_to_f32(T.wq[OB4]);
    for (int k = 0; k < HID; ++k) y += h3[i * HID + k] * bf16_to_f32(T.wq[OW4 + k]);
    const float res = i < B ? y - t[i] : 0.0f;
    T.dy[i] = 2.0f * res / (float)B;
    part += res * res;
  }
  red[tid] = part;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) T.loss[0] = red[0] / (float)B;
  // output layer gradients and dz_3 = (dy W4^T) * silu'(z_3)
  if (tid < HID) {
    float s = 0.0f;
    for (int i = 0; i < Bp; ++i) s += h3[i * HID + tid] * T.dy[i];
    T.grad[OW4 + tid] = s;
  } else if (tid == HID) {
    float s = 0.0f;
    for (int i = 0; i < Bp; ++i) s += T.dy[i];
    T.grad[OB4] = s;
  }
  {
    const float* z3 = T.z + (size_t)2 * MAXB * HID;
    for (int k = tid; k < Bp * HID; k += 256) {
      const int i = k / HID, c = k % HID;
      T.dz0[k] = T.dy[i] * bf16_to_f32(T.wq[OW4 + c]) * silu_grad(z3[k]);
    }
  }
  __syncthreads();
  float* dz = T.dz0;
  float* dzn = T.dz1;
  for (int l = 2; l >= 0; --l) {
    const int K = l == 0 ? 4 : HID;  // fan-in of layer l
    const float* hin = l == 0 ? T.xn : T.h + (size_t)(l - 1) * MAXB * HID;
    // grad W_l = h_{l-1}^T dz_l  [K x 64], contraction over the batch
    const int nti = l == 0 ? 1 : 4;
    for (int item = w; item < nti * 4; item += 4) {
      const int ti = item >> 2, tj = item & 3;
      v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
      acc = mfma_tile(
          Bp,
          [&](int i, int k) {
            const int a = 16 * ti + i;
            return a < K ? hin[k * K + a] : 0.0f;
          },
          [&](int k, int j) { return dz[k * HID + 16 * tj + j]; }, acc);
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * ti + 4 * q + v;
        if (a < K) T.grad[OW[l] + a * HID + 16 * tj + r] = acc[v];
      }
    }
    if (tid < HID) {
      float s = 0.0f;
      for (int i = 0; i < Bp; ++i) s += dz[i * HID + tid];
      T.grad[OB[l] + tid] = s;
    }
    if (l > 0) {
      // dz_{l-1} = (dz_l W_l^T) * silu'(z_{l-1})
      const float* zp = T.z + (size_t)(l - 1) * MAXB * HID;
      for (int item = w; item < ngroups * 4; item += 4) {
        const int g = item >> 2, jt = item & 3;
        v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = mfma_tile(
            HID, [&](int i, int k) { return dz[(16 * g + i) * HID + k]; },
            [&](int k, int j) { return bf16_to_f32(T.wq[OW[l] + (16 * jt + j) * HID + k]); }, acc);
        for (int v = 0; v < 4; ++v) {
          const int idx = (16 * g + 4 * q + v) * HID + 16 * jt + r;
          dzn[idx] = acc[v] * silu_grad(zp[idx]);
        }
      }
    }
    __syncthreads();
    float* tmp = dz;
    dz = dzn;
    dzn = tmp;
  }
  if (!update) return;
  // Adam with bias correction on the float32 masters, then the bf16 copy
  for (int p = tid; p < NP; p += 256) {
    const float g = T.grad[p];
    const float m = b1 * T.m[p] + (1.0f - b1) * g;
    const float v = b2 * T.v[p] + (1.0f - b2) * g * g;
    T.m[p] = m;
    T.v[p] = v;
    const float mh = m / bc1, vh = v / bc2;
    const float nw = T.master[p] - lr * mh / (sqrtf(vh) + eps);
    T.master[p] = nw;
    T.wq[p] = f32_to_bf16(nw);
  }
}

__global__ void k_mlp_init(float* master, uint16_t* wq, float* m, float* v, int np) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  wq[p] = f32_to_bf16(master[p]);
  m[p] = 0.0f;
  v[p] = 0.0f;
}

struct Bump {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

size_t mlp_layout(char* base, Train* T) {
  Bump b{base};
  Train t;
  t.master = b.take<float>(NP);
  t.m = b.take<float>(NP);
  t.v = b.take<float>(NP);
  t.grad = b.take<float>(NP);
  t.wq = b.take<uint16_t>(NP);
  t.loss = b.take<float>(1);
  t.xn = b.take<float>((size_t)MAXB * 4);
  t.z = b.take<float>((size_t)3 * MAXB * HID);
  t.h = b.take<float>((size_t)3 * MAXB * HID);
  t.dz0 = b.take<float>((size_t)MAXB * HID);
  t.dz1 = b.take<float>((size_t)MAXB * HID);
  t.dy = b.take<float>(MAXB);
  if (T) *T = t;
  return b.off + 256;
}

bool valid_cfg(const sdpdem_mlp_config* c) {
  if (!c) return false;
  for (int f = 0; f < 4; ++f)
    if (!(c->norm_std[f] > 0.0f) || !std::isfinite(c->norm_mean[f])) return false;
  if (!(c->lr > 0.0f) || !(c->beta1 >= 0.0f && c->beta1 < 1.0f) ||
      !(c->beta2 >= 0.0f && c->beta2 < 1.0f) || !(c->eps >= 0.0f))
    return false;
  return c->max_batch >= 1 && c->max_batch <= MAXB;
}

}  // namespace

struct sdpdem_mlp {
  sdpdem_mlp_config cfg;
  Train T;
  Norm nrm;
  int64_t steps = 0;
};

extern "C" {

int sdpdem_mlp_workspace_bytes(const sdpdem_mlp_config* cfg, size_t* bytes) {
  if (!bytes || !valid_cfg(cfg)) return SDPDEM_E_INVALID_ARG;
  *bytes = mlp_layout(nullptr, nullptr);
  return SDPDEM_OK;
}

int sdpdem_mlp_create(const sdpdem_mlp_config* cfg, const float* init_params, void* d_workspace,
                      size_t workspace_bytes, void* hip_stream, sdpdem_mlp** out) {
  if (!out) return SDPDEM_E_INVALID_ARG;
  *out = nullptr;
  if (!valid_cfg(cfg) || !init_params || !d_workspace) return SDPDEM_E_INVALID_ARG;
  char* base = reinterpret_cast<char*>(((uintptr_t)d_workspace + 255) & ~(uintptr_t)255);
  const size_t need = mlp_layout(nullptr, nullptr);
  if (workspace_bytes < need || (size_t)(base - (char*)d_workspace) + need - 256 > workspace_bytes)
    return SDPDEM_E_WORKSPACE_TOO_SMALL;
  sdpdem_mlp* m = new (std::nothrow) sdpdem_mlp();
  if (!m) return SDPDEM_E_INVALID_ARG;
  m->cfg = *cfg;
  mlp_layout(base, &m->T);
  for (int f = 0; f < 4; ++f) {
    m->nrm.mean[f] = cfg->norm_mean[f];
    m->nrm.inv_std[f] = 1.0f / cfg->norm_std[f];
  }
  hipStream_t st = (hipStream_t)hip_stream;
  bool ok = hipMemcpyAsync(m->T.master, init_params, sizeof(float) * NP, hipMemcpyHostToDevice,
                           st) == hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (ok) {
    k_mlp_init<<<(NP + 255) / 256, 256, 0, st>>>(m->T.master, m->T.wq, m->T.m, m->T.v, NP);
    ok = hipStreamSynchronize(st) == hipSuccess && hipGetLastError() == hipSuccess;
  }
  if (!ok) {
    delete m;
    return SDPDEM_E_HIP;
  }
  *out = m;
  return SDPDEM_OK;
}

int sdpdem_mlp_predict(sdpdem_mlp* m, const float* d_x, float* d_y, int64_t n, void* hip_stream) {
  if (!m || n < 0 || (n > 0 && (!d_x || !d_y))) return SDPDEM_E_INVALID_ARG;
  if (n == 0) return SDPDEM_OK;
  // enough blocks to fill the chip; each wavefront walks its 16-row groups
  const int64_t groups = (n + 15) / 16;
  const int64_t blocks = std::min<int64_t>((groups + PRED_WAVES - 1) / PRED_WAVES, 2048);
  const int64_t per_wave = (groups + blocks * PRED_WAVES - 1) / (blocks * PRED_WAVES);
  k_mlp_predict<<<(unsigned)blocks, 64 * PRED_WAVES, 0, (hipStream_t)hip_stream>>>(
      m->T.wq, m->nrm, d_x, d_y, n, per_wave);
  return hipGetLastError() == hipSuccess ? SDPDEM_OK : SDPDEM_E_HIP;
}

int sdpdem_mlp_train_step(sdpdem_mlp* m, const float* d_x, const float* d_t, int32_t batch,
                          int32_t update, void* hip_stream) {
  if (!m || !d_x || !d_t || batch < 1 || batch > m->cfg.max_batch) return SDPDEM_E_INVALID_ARG;
  float bc1 = 1.0f, bc2 = 1.0f;
  if (update) {
    m->steps += 1;
    bc1 = (float)(1.0 - std::pow((double)m->cfg.beta1, (double)m->steps));
    bc2 = (float)(1.0 - std::pow((double)m->cfg.beta2, (double)m->steps));
  }
  k_mlp_train<<<1, 256, 0, (hipStream_t)hip_stream>>>(m->T, m->nrm, d_x, d_t, batch, update ? 1 : 0,
                                                     m->cfg.lr, m->cfg.beta1, m->cfg.beta2,
                                                     m->cfg.eps, bc1, bc2);
  return hipGetLastError() == hipSuccess ? SDPDEM_OK : SDPDEM_E_HIP;
}

int sdpdem_mlp_read(sdpdem_mlp* m, float* params, float* used_params, float* grad, float* loss,
                    int64_t* steps, void* hip_stream) {
  if (!m) return SDPDEM_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<uint16_t> q;
  bool ok = true;
  if (params)
    ok = ok && hipMemcpyAsync(params, m->T.master, sizeof(float) * NP, hipMemcpyDeviceToHost,
                              st) == hipSuccess;
  if (used_params) {
    q.resize(NP);
    ok = ok && hipMemcpyAsync(q.data(), m->T.wq, sizeof(uint16_t) * NP, hipMemcpyDeviceToHost,
                              st) == hipSuccess;
  }
  if (grad)
    ok = ok && hipMemcpyAsync(grad, m->T.grad, sizeof(float) * NP, hipMemcpyDeviceToHost, st) ==
                   hipSuccess;
  if (loss)
    ok = ok && hipMemcpyAsync(loss, m->T.loss, sizeof(float), hipMemcpyDeviceToHost, st) ==
                   hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) return SDPDEM_E_HIP;
  if (used_params)
    for (int p = 0; p < NP; ++p) {
      uint32_t u = (uint32_t)q[(size_t)p] << 16;
      std::memcpy(&used_params[p], &u, sizeof(float));
    }
  if (steps) *steps = m->steps;
  return SDPDEM_OK;
}

void sdpdem_mlp_destroy(sdpdem_mlp* m) { delete m; }

}  // extern "C"
