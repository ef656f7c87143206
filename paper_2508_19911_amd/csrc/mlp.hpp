// mlp.hpp -- troubled-cell indicator network on gfx950 matrix cores.
//
// The learned form of the GENO switch: a cell whose logit exceeds the threshold runs the full
// nonlinear GENO reconstruction, the others take the linear P^4 (both from arXiv 2508.19911,
// Sec. 3.2).  Network: 64 inputs (59 used) -> 32 -> 32 -> 32 -> 1, ReLU, logit output.
//   * inputs: for rho and rho E, along x, y, z: Q(i+o) - Q(i) for o = -2,-1,1,2 and h dQ/dx of the
//     cells o = -2..2, divided by s = max|difference| + max|h dQ| + 1e-12 |Q(i)|; then for each of
//     the 5 variables log10(max |difference or h dQ| on those lines / (h_max sqrt(S_v))), the
//     variation against the GENO smoothness floor (clipped below at -12);
//   * forward: hidden layers on v_mfma_f32_16x16x16_bf16 (bf16 inputs and weights, fp32
//     accumulation), bias + ReLU in fp32, h1 and h2 rounded to bf16 for the next layer, h3 kept in
//     fp32 for the final dot product with w4;
//   * backward: the same forward, then fp32 matrix cores (v_mfma_f32_16x16x4_f32) for the weight
//     gradients and the back-propagated deltas (through the bf16-rounded weights);
//   * Adam with fp32 master weights, minibatches of 1024 visited in a seeded affine permutation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace cgks {
namespace mlp {

constexpr int NIN = 64, NH = 32, NPARAM = 4225;
constexpr int OW1 = 0, OB1 = 2048, OW2 = 2080, OB2 = 3104, OW3 = 3136, OB3 = 4160, OW4 = 4192,
              OB4 = 4224;
constexpr int BATCH = 1024;
constexpr int WAVES_PER_BATCH = BATCH / 64;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// workspace: params | adam m | adam v | per-wave gradient partials | loss partials | grad accumulator
constexpr size_t OFF_PARAMS = 0;
constexpr size_t OFF_M = 4352 * 4;
constexpr size_t OFF_V = 2 * 4352 * 4;
constexpr size_t OFF_PART = 3 * 4352 * 4;
constexpr size_t OFF_LOSS = OFF_PART + (size_t)WAVES_PER_BATCH * 4352 * 4;
constexpr size_t OFF_GACC = OFF_LOSS + 4096;
constexpr size_t OFF_END = OFF_GACC + 4352 * 8;
inline size_t workspace_bytes() { return (OFF_END + 255) & ~size_t(255); }

// float -> bf16 bits, round to nearest even: one hardware conversion on gfx950 (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------- features
// The 64 features of one cell, each handed to put(n, value) as soon as it is known (no 64-entry
// array stays live in registers).
template <class T, class Put>
__device__ __forceinline__ void cell_features(const Grid& g, const double* __restrict__ Q,
                                              const T* __restrict__ G, int cell, Put&& put) {
  int i, j, k;
  i = cell % g.nx;
  const int jk = cell / g.nx;
  j = jk % g.ny;
  k = jk / g.ny;
  const long long N = g.N;
  // byte offsets of the line cells o = -2..2 along each axis, in planes of double and of T
  uint32_t oq[3][5], og[3][5];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
      const int ii = d == 0 ? wrap_o(i, o, g.nx) : i;
      const int jj = d == 1 ? wrap_o(j, o, g.ny) : j;
      const int kk = d == 2 ? wrap_o(k, o, g.nz) : k;
      const uint32_t c = (uint32_t)((kk * g.ny + jj) * g.nx + ii);
      oq[d][o + 2] = c * 8u;
      og[d][o + 2] = c * (uint32_t)sizeof(T);
    }
  double q5[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) q5[v] = Q[v * N + cell];
  double mx_line[2];  // the maximum of feature 54 + v for v = 0, 4, found on the way
#pragma unroll
  for (int vi = 0; vi < 2; ++vi) {
    const int v = vi ? 4 : 0;
    const BufPlane<double> qv(Q + v * N, N);
    const double q0 = q5[v];
    double dv[3][4], gv[3][5];
    double mxd = 0.0, mxg = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const BufPlane<T> gd(G + (d * 5 + v) * N, N);
#pragma unroll
      for (int o = -2; o <= 2; ++o) {
        if (o != 0) {
          const double dd = qv(oq[d][o + 2]) - q0;
          dv[d][o < 0 ? o + 2 : o + 1] = dd;
          mxd = fmax(mxd, fabs(dd));
        }
        const double gg = g.h[d] * double(gd(og[d][o + 2]));
        gv[d][o + 2] = gg;
        mxg = fmax(mxg, fabs(gg));
      }
    }
    mx_line[vi] = fmax(mxd, mxg);
    const double is = 1.0 / (mxd + mxg + 1e-12 * fabs(q0));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
      for (int m = 0; m < 4; ++m) put(vi * 27 + d * 9 + m, float(dv[d][m] * is));
#pragma unroll
      for (int m = 0; m < 5; ++m) put(vi * 27 + d * 9 + 4 + m, float(gv[d][m] * is));
    }
  }
  // features 54..58: per conservative variable, log10 of the largest difference or h dQ on the same
  // lines over h_max sqrt(S_v), S_v the variable's GENO scale (clipped below at -12)
  const double hmax = fmax(g.h[0], fmax(g.h[1], g.h[2]));
#pragma unroll 1
  for (int v = 0; v < 5; ++v) {
    double mx = v == 0 ? mx_line[0] : mx_line[1];
    if (v != 0 && v != 4) {  // the momenta: their lines were not read above
      const BufPlane<double> qv(Q + v * N, N);
      mx = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const BufPlane<T> gd(G + (d * 5 + v) * N, N);
#pragma unroll
        for (int o = 0; o < 5; ++o) {
          mx = fmax(mx, fabs(qv(oq[d][o]) - q5[v]));
          mx = fmax(mx, fabs(g.h[d] * double(gd(og[d][o]))));
        }
      }
    }
    // the ratio in FP64, its logarithm in FP32 (a feature needs no more)
    put(54 + v, fmaxf(log10f(float(mx / (hmax * sqrt(geno_scale(q5, v))))), -12.0f));
  }
#pragma unroll
  for (int n = 59; n < 64; ++n) put(n, 0.0f);
}

template <class T>
__global__ __launch_bounds__(256) void k_features(Grid g, const double* __restrict__ Q,
                                                  const T* __restrict__ G, float* __restrict__ out) {
  const int cell = blockIdx.x * 256 + threadIdx.x;
  if (cell >= g.N) return;
  float* o = out + (long long)cell * 64;
  cell_features<T>(g, Q, G, cell, [&](int n, float x) { o[n] = x; });
}

template <class T>
int launch_features(const Grid& g, const double* Q, const T* G, float* out, hipStream_t s) {
  k_features<T><<<(unsigned)((g.N + 255) / 256), 256, 0, s>>>(g, Q, G, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ---------------------------------------------------------------------------- GENO labels
template <class T>
__global__ __launch_bounds__(256) void k_labels(Grid g, const double* __restrict__ Q,
                                                const T* __restrict__ G, GenoParams gp, double thr,
                                                unsigned char* __restrict__ out) {
  const int cell = blockIdx.x * 256 + threadIdx.x;
  if (cell >= g.N) return;
  int i = cell % g.nx;
  const int jk = cell / g.nx;
  int j = jk % g.ny, k = jk / g.ny;
  const long long N = g.N;
  uint32_t oq[tab::NSTEN], og[tab::NSTEN];
#pragma unroll
  for (int s = 0; s < tab::NSTEN; ++s) {
    const uint32_t c = (uint32_t)((wrap_o(k, tab::SOFF[s][2], g.nz) * g.ny + wrap_o(j, tab::SOFF[s][1], g.ny)) *
                                      g.nx + wrap_o(i, tab::SOFF[s][0], g.nx));
    oq[s] = c * 8u;
    og[s] = c * (uint32_t)sizeof(T);
  }
  double worst = 0.0;
  double q5[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) q5[v] = Q[v * N + cell];
#pragma unroll 1
  for (int v = 0; v < 5; ++v) {
    const BufPlane<double> qa(Q + v * N, N);
    const BufPlane<T> ga[3] = {BufPlane<T>(G + v * N, N), BufPlane<T>(G + (5 + v) * N, N),
                               BufPlane<T>(G + (10 + v) * N, N)};
    T a[tab::NB], dface[6], g0[3];
#pragma unroll
    for (int m = 0; m < tab::NB; ++m) a[m] = T(0);
    gather_coefficients<T>(g, qa, ga, oq, og, q5[v], a, dface, g0);
    const T chi = geno_blend(dface, g0, a, gp, data<T>(gp.eps + gp.hmax2 * geno_scale(q5, v)));
    worst = fmax(worst, fabs(1.0 - double(chi)));
  }
  out[cell] = worst > thr ? 1 : 0;
}

template <class T>
int launch_labels(const Grid& g, const double* Q, const T* G, const GenoParams& gp, double thr,
                  unsigned char* out, hipStream_t s) {
  k_labels<T><<<(unsigned)((g.N + 255) / 256), 256, 0, s>>>(g, Q, G, gp, thr, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ---------------------------------------------------------------------------- forward (one wave)
// xs: 64 x 64 bf16 (row = sample) in LDS; h1: 64 x 32 bf16; w: bf16 W1|W2|W3 in LDS.
// On return, z[mt][nt] holds layer-3 pre-activations; z1/z2 (optional) keep layers 1 and 2.
// Inference staging of one wave: rows padded by 4 bf16 (8 bytes), so the 16 rows an MFMA operand load
// touches fall on different LDS banks, and every 4-element operand is one aligned 8-byte access.
constexpr int XS = 64 + 4, HS = 32 + 4;
struct alignas(16) WaveLDS {
  uint16_t x[64 * XS];   // features, then each hidden layer in turn (row stride HS)
};

__device__ __forceinline__ f32x4 mfma_bf16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// One dense layer Y = X W^T + b on the wave's 64 rows: X [64][K] bf16 (row stride XR), W [32][K]
// bf16 (row stride WR), result tile (mt, nt) in acc[mt][nt] (lane: rows 4(l/16)+r, column l%16).
// Both strides keep every 4-element operand 8-byte aligned.
template <int K, int XR = K, int WR = K>
__device__ __forceinline__ void dense_bf16(const uint16_t* X, const uint16_t* W, const float* bias,
                                           f32x4 acc[4][2]) {
  static_assert(XR % 4 == 0 && WR % 4 == 0, "8-byte operand rows");
  const int l = threadIdx.x & 63;
  const int r16 = l & 15, q = l >> 4;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const float b = bias[nt * 16 + r16];
      acc[mt][nt] = f32x4{b, b, b, b};
    }
#pragma unroll
  for (int kt = 0; kt < K / 16; ++kt) {
    bf16x4 bw[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
      bw[nt] = *reinterpret_cast<const bf16x4*>(W + (nt * 16 + r16) * WR + kt * 16 + 4 * q);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const bf16x4 a = *reinterpret_cast<const bf16x4*>(X + (mt * 16 + r16) * XR + kt * 16 + 4 * q);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = mfma_bf16(a, bw[nt], acc[mt][nt]);
    }
  }
}

// ReLU of a layer result, rounded to bf16, stored row-major [64][32] (row stride HR) in LDS
template <int HR = 32>
__device__ __forceinline__ void store_relu_bf16(const f32x4 acc[4][2], uint16_t* H) {
  const int l = threadIdx.x & 63;
  const int r16 = l & 15, q = l >> 4;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float z = acc[mt][nt][r];
        H[(mt * 16 + 4 * q + r) * HR + nt * 16 + r16] = f2bf(z > 0.0f ? z : 0.0f);
      }
}

// logits of the wave's 64 rows from the layer-3 accumulators: sum_n w4[n] relu(z3) + b4
__device__ __forceinline__ void logits_from_z3(const f32x4 z3[4][2], const float* w4, float b4,
                                               float out[4][4]) {
  const int l = threadIdx.x & 63;
  const int r16 = l & 15;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float s = 0.0f;
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const float z = z3[mt][nt][r];
        s += (z > 0.0f ? z : 0.0f) * w4[nt * 16 + r16];
      }
      // sum over the 16 lanes holding the 16 columns of this row group
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      out[mt][r] = s + b4;
    }
}

// ---------------------------------------------------------------------------- inference
template <class T>
__global__ __launch_bounds__(256, 3) void k_infer(Grid g, const double* __restrict__ Q,
                                               const T* __restrict__ G,
                                               const float* __restrict__ params,
                                               unsigned char* __restrict__ flags,
                                               float* __restrict__ logits, float thr,
                                               const double* __restrict__ ctl) {
  if (ctl && ctl[1] != 0.0) return;  // the step was stopped (see k_step_control)
  __shared__ WaveLDS wl[4];
  // bf16 weights, rows padded like the activations: W1 [32][XS], W2 and W3 [32][HS]
  constexpr int OWS2 = 32 * XS, OWS3 = OWS2 + 32 * HS, NWS = OWS3 + 32 * HS;
  __shared__ alignas(16) uint16_t wsh[NWS];
  __shared__ float bsh[3 * 32 + 32 + 1];
  {
    // every load of the staging first (16-byte loads: W1 is 512 of them, W2 and W3 256 each, all
    // 16-byte aligned), then the conversions and LDS stores; a loop that stored each weight before
    // loading the next waited for every load in turn
    const int t = (int)threadIdx.x & 255;
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4* p4 = reinterpret_cast<const f4*>(params);
    static_assert(OW1 % 4 == 0 && OW2 % 4 == 0 && OW3 % 4 == 0, "16-byte weight rows");
    const f4 a0 = p4[OW1 / 4 + t], a1 = p4[OW1 / 4 + 256 + t], b = p4[OW2 / 4 + t], c = p4[OW3 / 4 + t];
    float bias[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (t < 32) {
      bias[0] = params[OB1 + t];
      bias[1] = params[OB2 + t];
      bias[2] = params[OB3 + t];
      bias[3] = params[OW4 + t];
    }
    const float b4 = t == 0 ? params[OB4] : 0.0f;
    auto put4 = [&](int off, const f4& x) {
      *reinterpret_cast<bf16x4*>(wsh + off) = bf16x4{(short)f2bf(x[0]), (short)f2bf(x[1]), (short)f2bf(x[2]), (short)f2bf(x[3])};
    };
    // element n = 4 (t or 256 + t) of W1 sits in row n / 64 at column n % 64; of W2, W3 row n / 32
    put4(((4 * t) >> 6) * XS + ((4 * t) & 63), a0);
    put4(((4 * (256 + t)) >> 6) * XS + ((4 * (256 + t)) & 63), a1);
    put4(OWS2 + ((4 * t) >> 5) * HS + ((4 * t) & 31), b);
    put4(OWS3 + ((4 * t) >> 5) * HS + ((4 * t) & 31), c);
    if (t < 32) {
      bsh[t] = bias[0];
      bsh[32 + t] = bias[1];
      bsh[64 + t] = bias[2];
      bsh[96 + t] = bias[3];
    }
    if (t == 0) bsh[128] = b4;
  }
  static_assert(XS % 4 == 0 && HS % 4 == 0 && OWS2 % 4 == 0 && OWS3 % 4 == 0, "8-byte aligned weight rows");
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int base = blockIdx.x * 256 + w * 64;
  const int cell = base + l;
  {
    uint16_t* row = wl[w].x + l * XS;
    if (cell < g.N)
      cell_features<T>(g, Q, G, cell, [&](int n, float x) { row[n] = f2bf(x); });
    else
#pragma unroll
      for (int n = 0; n < 64; n += 4) *reinterpret_cast<bf16x4*>(row + n) = bf16x4{0, 0, 0, 0};
  }
  __syncthreads();
  f32x4 acc[4][2];
  // each layer's output overwrites its input rows in place (the rows are the wave's own, and a wave's
  // LDS operations complete in issue order, so the stores follow every load of the layer).  One row
  // buffer per wave instead of two brings the block to 44 KB of LDS and three waves per SIMD: 1.74 ->
  // 1.38 ms per launch at 256^3.
  dense_bf16<64, XS, XS>(wl[w].x, wsh, bsh, acc);
  store_relu_bf16<HS>(acc, wl[w].x);
  dense_bf16<32, HS, HS>(wl[w].x, wsh + OWS2, bsh + 32, acc);
  store_relu_bf16<HS>(acc, wl[w].x);
  dense_bf16<32, HS, HS>(wl[w].x, wsh + OWS3, bsh + 64, acc);
  float z[4][4];
  logits_from_z3(acc, bsh + 96, bsh[128], z);
  if ((l & 15) == 0) {
    const int q = l >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = base + mt * 16 + 4 * q + r;
        if (c < g.N) {
          if (flags) flags[c] = z[mt][r] > thr ? 1 : 0;
          if (logits) logits[c] = z[mt][r];
        }
      }
  }
}

template <class T>
int launch_infer(const Grid& g, const double* Q, const T* G, const float* params,
                 unsigned char* flags, float* logits, double thr, char* /*ws*/, hipStream_t s,
                 const double* ctl = nullptr) {
  k_infer<T><<<(unsigned)((g.N + 255) / 256), 256, 0, s>>>(g, Q, G, params, flags, logits, (float)thr, ctl);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ---------------------------------------------------------------------------- training step
struct alignas(16) TrainLDS {
  uint16_t x[64 * 64];
  float z1[64 * 32];
  uint16_t h1[64 * 32];
  float z2[64 * 32];
  uint16_t h2[64 * 32];
  float dz[64 * 32];  // delta of the current layer, row = sample
  float dh[64 * 32];
  float zl[64];
  uint16_t wb[32 * 64 + 2 * 32 * 32];
};

__device__ __forceinline__ uint32_t sample_index(long long b, uint64_t pa, uint64_t pb, long long n) {
  return (uint32_t)((pa * (uint64_t)b + pb) % (uint64_t)n);
}

// One wave = 64 samples of the minibatch; writes the wave's gradient partial (sum over its
// samples of d loss_s / d params, loss scaled by inv_count) and its loss sum.
__global__ __launch_bounds__(64) void k_train_grad(const float* __restrict__ params,
                                                   const uint16_t* __restrict__ X,
                                                   const float* __restrict__ Y, long long n,
                                                   long long b0, long long count, uint64_t pa,
                                                   uint64_t pb, float inv_count,
                                                   float* __restrict__ part,
                                                   float* __restrict__ loss_part) {
  __shared__ TrainLDS s;
  const int l = threadIdx.x;
  const int r16 = l & 15, q = l >> 4;
  for (int t = l; t < 32 * 64 + 2 * 32 * 32; t += 64)
    s.wb[t] = f2bf(params[t < 2048 ? t : (t < 3072 ? OW2 + t - 2048 : OW3 + t - 3072)]);
  const long long bi = b0 + (long long)blockIdx.x * 64 + l;
  const bool valid = bi < b0 + count;
  const uint32_t si = valid ? sample_index(bi, pa, pb, n) : 0;
  for (int c = 0; c < 64; ++c) s.x[l * 64 + c] = valid ? X[(long long)si * 64 + c] : (uint16_t)0;
  const float y = valid ? Y[si] : 0.0f;
  __syncthreads();
  // forward
  f32x4 acc[4][2];
  dense_bf16<64>(s.x, s.wb, params + OB1, acc);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) s.z1[(mt * 16 + 4 * q + r) * 32 + nt * 16 + r16] = acc[mt][nt][r];
  store_relu_bf16(acc, s.h1);
  __syncthreads();
  dense_bf16<32>(s.h1, s.wb + 2048, params + OB2, acc);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) s.z2[(mt * 16 + 4 * q + r) * 32 + nt * 16 + r16] = acc[mt][nt][r];
  store_relu_bf16(acc, s.h2);
  __syncthreads();
  dense_bf16<32>(s.h2, s.wb + 3072, params + OB3, acc);
  // z3 -> s.dh (temporarily), logits
  float zz[4][4];
  logits_from_z3(acc, params + OW4, params[OB4], zz);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) s.dh[(mt * 16 + 4 * q + r) * 32 + nt * 16 + r16] = acc[mt][nt][r];
  if (r16 == 0)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) s.zl[mt * 16 + 4 * q + r] = zz[mt][r];
  __syncthreads();
  // loss and output delta (row l = this lane's sample)
  const float z = s.zl[l];
  float lossv = 0.0f, dzl = 0.0f;
  if (valid) {
    lossv = fmaxf(z, 0.0f) - y * z + log1pf(expf(-fabsf(z)));
    dzl = (1.0f / (1.0f + expf(-z)) - y) * inv_count;
  }
  // w4, b4 gradients and layer-3 delta
  float* gp = part + (long long)blockIdx.x * 4352;
  {
    // dW4[n] = sum_s dzl_s relu(z3[s][n]); delta3[s][n] = dzl_s w4[n] [z3 > 0]
    for (int nn = 0; nn < 32; ++nn) {
      const float z3 = s.dh[l * 32 + nn];
      float v = z3 > 0.0f ? dzl * z3 : 0.0f;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (l == 0) gp[OW4 + nn] = v;
    }
    float v = dzl;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (l == 0) gp[OB4] = v;
    float lv = lossv;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lv += __shfl_xor(lv, off, 64);
    if (l == 0) loss_part[blockIdx.x] = lv;
    for (int nn = 0; nn < 32; ++nn) {
      const float z3 = s.dh[l * 32 + nn];
      s.dz[l * 32 + nn] = z3 > 0.0f ? dzl * params[OW4 + nn] : 0.0f;
    }
  }
  __syncthreads();
  // three backward layers: (delta, H_in, W, K_in, offsets)
#pragma unroll 1
  for (int layer = 3; layer >= 1; --layer) {
    const int K = layer == 1 ? 64 : 32;
    const uint16_t* Hin = layer == 3 ? s.h2 : (layer == 2 ? s.h1 : s.x);
    const uint16_t* Wl = layer == 3 ? s.wb + 3072 : (layer == 2 ? s.wb + 2048 : s.wb);
    const int oW = layer == 3 ? OW3 : (layer == 2 ? OW2 : OW1);
    const int oB = layer == 3 ? OB3 : (layer == 2 ? OB2 : OB1);
    // dW[j][k] = sum_s dz[s][j] H[s][k]  (M = j (32), N = k (K), K-dim = samples (64))
    for (int nt = 0; nt < K / 16; ++nt) {
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        f32x4 c = f32x4{0, 0, 0, 0};
#pragma unroll 4
        for (int kt = 0; kt < 16; ++kt) {
          const int sm = kt * 4 + q;
          const float a = s.dz[sm * 32 + mt * 16 + r16];
          const float b = bf2f(Hin[sm * K + nt * 16 + r16]);
          c = mfma_f32(a, b, c);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) gp[oW + (mt * 16 + 4 * q + r) * K + nt * 16 + r16] = c[r];
      }
    }
    // db[j] = sum_s dz[s][j]
    if (l < 32) {
      float v = 0.0f;
      for (int sm = 0; sm < 64; ++sm) v += s.dz[sm * 32 + l];
      gp[oB + l] = v;
    }
    if (layer == 1) break;
    // dh[s][k] = sum_j dz[s][j] W[j][k], then the ReLU mask of the layer below
    const float* zb = layer == 3 ? s.z2 : s.z1;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        f32x4 c = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int kt = 0; kt < 8; ++kt) {
          const float a = s.dz[(mt * 16 + r16) * 32 + kt * 4 + q];
          const float b = bf2f(Wl[(kt * 4 + q) * 32 + nt * 16 + r16]);
          c = mfma_f32(a, b, c);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = mt * 16 + 4 * q + r, col = nt * 16 + r16;
          s.dh[row * 32 + col] = zb[row * 32 + col] > 0.0f ? c[r] : 0.0f;
        }
      }
    __syncthreads();
    for (int t = l; t < 64 * 32; t += 64) s.dz[t] = s.dh[t];
    __syncthreads();
  }
}

// sum the wave partials (fixed order) into g and apply Adam (or accumulate into gacc)
__global__ __launch_bounds__(256) void k_reduce_adam(float* __restrict__ params, float* __restrict__ m,
                                                     float* __restrict__ v,
                                                     const float* __restrict__ part, int nwaves,
                                                     float lr, float bc1, float bc2,
                                                     double* __restrict__ gacc, int mode) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= NPARAM) return;
  float g = 0.0f;
  for (int w = 0; w < nwaves; ++w) g += part[(long long)w * 4352 + p];
  if (mode == 1) {
    gacc[p] += (double)g;
    return;
  }
  const float b1 = 0.9f, b2 = 0.999f;
  const float mm = b1 * m[p] + (1.0f - b1) * g;
  const float vv = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  params[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
}

inline uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
inline uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

inline int train(char* ws, const uint16_t* X, const float* Y, long n, int epochs, double lr,
                 uint64_t seed, double* final_loss, hipStream_t s) {
  float* params = reinterpret_cast<float*>(ws + OFF_PARAMS);
  float* m = reinterpret_cast<float*>(ws + OFF_M);
  float* v = reinterpret_cast<float*>(ws + OFF_V);
  float* part = reinterpret_cast<float*>(ws + OFF_PART);
  float* lpart = reinterpret_cast<float*>(ws + OFF_LOSS);
  if (hipMemsetAsync(m, 0, 2 * 4352 * 4, s) != hipSuccess) return -3;
  uint64_t st = seed;
  long step = 0;
  double last = 0.0;
  std::vector<float> lh(WAVES_PER_BATCH);
  for (int ep = 0; ep < epochs; ++ep) {
    uint64_t pa = splitmix(st) % (uint64_t)n;
    while (gcd64(pa, (uint64_t)n) != 1) pa = (pa + 1) % (uint64_t)n;
    if (n == 1) pa = 1;
    const uint64_t pb = splitmix(st) % (uint64_t)n;
    double esum = 0.0;
    for (long long b0 = 0; b0 < n; b0 += BATCH) {
      const long long cnt = (n - b0 < BATCH) ? n - b0 : BATCH;
      const int nw = (int)((cnt + 63) / 64);
      k_train_grad<<<nw, 64, 0, s>>>(params, X, Y, n, b0, cnt, pa, pb, 1.0f / (float)cnt, part, lpart);
      ++step;
      const float bc1 = 1.0f - powf(0.9f, (float)step), bc2 = 1.0f - powf(0.999f, (float)step);
      k_reduce_adam<<<(NPARAM + 255) / 256, 256, 0, s>>>(params, m, v, part, nw, (float)lr, bc1, bc2,
                                                         nullptr, 0);
      if (hipGetLastError() != hipSuccess) return -3;
      if (ep == epochs - 1) {
        if (hipMemcpyAsync(lh.data(), lpart, nw * 4, hipMemcpyDeviceToHost, s) != hipSuccess) return -3;
        if (hipStreamSynchronize(s) != hipSuccess) return -3;
        for (int w = 0; w < nw; ++w) esum += lh[w];
      }
    }
    if (ep == epochs - 1) last = esum / (double)n;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return -3;
  *final_loss = last;
  return 0;
}

// gradient of the mean loss over all n samples (in order), host output
inline int loss_grad(char* ws, const uint16_t* X, const float* Y, long n, double* loss, double* grad,
                     hipStream_t s) {
  float* params = reinterpret_cast<float*>(ws + OFF_PARAMS);
  float* part = reinterpret_cast<float*>(ws + OFF_PART);
  float* lpart = reinterpret_cast<float*>(ws + OFF_LOSS);
  double* gacc = reinterpret_cast<double*>(ws + OFF_GACC);
  if (hipMemsetAsync(gacc, 0, 4352 * 8, s) != hipSuccess) return -3;
  double lsum = 0.0;
  std::vector<float> lh(WAVES_PER_BATCH);
  for (long long b0 = 0; b0 < n; b0 += BATCH) {
    const long long cnt = (n - b0 < BATCH) ? n - b0 : BATCH;
    const int nw = (int)((cnt + 63) / 64);
    k_train_grad<<<nw, 64, 0, s>>>(params, X, Y, n, b0, cnt, 1, 0, 1.0f / (float)n, part, lpart);
    k_reduce_adam<<<(NPARAM + 255) / 256, 256, 0, s>>>(params, nullptr, nullptr, part, nw, 0.0f, 1.0f,
                                                       1.0f, gacc, 1);
    if (hipGetLastError() != hipSuccess) return -3;
    if (hipMemcpyAsync(lh.data(), lpart, nw * 4, hipMemcpyDeviceToHost, s) != hipSuccess) return -3;
    if (hipStreamSynchronize(s) != hipSuccess) return -3;
    for (int w = 0; w < nw; ++w) lsum += lh[w];
  }
  if (hipMemcpyAsync(grad, gacc, NPARAM * 8, hipMemcpyDeviceToHost, s) != hipSuccess) return -3;
  if (hipStreamSynchronize(s) != hipSuccess) return -3;
  *loss = lsum / (double)n;
  return 0;
}

}  // namespace mlp
}  // namespace cgks
