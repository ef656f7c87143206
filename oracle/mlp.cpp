/*
 * mlp.cpp -- oracle: troubled-cell indicator network, forward pass and the gradient of the
 * binary cross-entropy.  TEST INFRASTRUCTURE ONLY.
 *
 * The indicator is not part of the paper; it is the learned form asked for alongside the
 * method (reading R17): 64 inputs (59 used) -> 32 -> 32 -> 32 -> 1, ReLU hidden layers, a
 * logit output.  Parameter layout (float): W1[32][64], b1[32], W2[32][32], b2[32], W3[32][32],
 * b3[32], w4[32], b4.  With bf16 emulation on, the inputs of the three hidden layers (x, h1,
 * h2) and their weights are rounded to bfloat16 (nearest even), matching BF16 matrix-core
 * inputs with wider accumulation; h3, w4 and the biases stay unrounded.  Arithmetic is FP64.
 */
#include "oracle_internal.h"

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace cgkso {

static double bf16(double v) {
  float f = static_cast<float>(v);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return f;  // inf / nan unchanged
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  std::memcpy(&f, &u, 4);
  return f;
}

struct Net {
  double W1[32][64], b1[32], W2[32][32], b2[32], W3[32][32], b3[32], w4[32], b4;
};

static void load(const float* p, int r, Net& n) {
  auto R = [&](float v) { return r ? bf16(v) : static_cast<double>(v); };
  int o = 0;
  for (int j = 0; j < 32; ++j)
    for (int k = 0; k < 64; ++k) n.W1[j][k] = R(p[o++]);
  for (int j = 0; j < 32; ++j) n.b1[j] = p[o++];
  for (int j = 0; j < 32; ++j)
    for (int k = 0; k < 32; ++k) n.W2[j][k] = R(p[o++]);
  for (int j = 0; j < 32; ++j) n.b2[j] = p[o++];
  for (int j = 0; j < 32; ++j)
    for (int k = 0; k < 32; ++k) n.W3[j][k] = R(p[o++]);
  for (int j = 0; j < 32; ++j) n.b3[j] = p[o++];
  for (int j = 0; j < 32; ++j) n.w4[j] = p[o++];
  n.b4 = p[o++];
}

struct Acts {
  double x[64], z1[32], h1[32], z2[32], h2[32], z3[32], h3[32], z4;
};

static void forward_one(const Net& n, const float* xin, int r, Acts& a) {
  auto R = [&](double v) { return r ? bf16(v) : v; };
  for (int k = 0; k < 64; ++k) a.x[k] = R(xin[k]);
  for (int j = 0; j < 32; ++j) {
    double s = n.b1[j];
    for (int k = 0; k < 64; ++k) s += n.W1[j][k] * a.x[k];
    a.z1[j] = s;
    a.h1[j] = R(s > 0.0 ? s : 0.0);
  }
  for (int j = 0; j < 32; ++j) {
    double s = n.b2[j];
    for (int k = 0; k < 32; ++k) s += n.W2[j][k] * a.h1[k];
    a.z2[j] = s;
    a.h2[j] = R(s > 0.0 ? s : 0.0);
  }
  for (int j = 0; j < 32; ++j) {
    double s = n.b3[j];
    for (int k = 0; k < 32; ++k) s += n.W3[j][k] * a.h2[k];
    a.z3[j] = s;
    a.h3[j] = s > 0.0 ? s : 0.0;
  }
  double s = n.b4;
  for (int k = 0; k < 32; ++k) s += n.w4[k] * a.h3[k];
  a.z4 = s;
}

void mlp_forward(const float* params, const float* x, long n, int bf, double* logits) {
  Net net;
  load(params, bf, net);
#pragma omp parallel for
  for (long i = 0; i < n; ++i) {
    Acts a;
    forward_one(net, x + i * 64, bf, a);
    logits[i] = a.z4;
  }
}

}  // namespace cgkso

using namespace cgkso;

extern "C" {

void cgkso_mlp_forward(const float* params, const float* x, long n, int bf16, double* logits) {
  mlp_forward(params, x, n, bf16, logits);
}

double cgkso_mlp_loss_grad(const float* params, const float* x, const float* y, long n, int bf,
                           double* grad) {
  Net net;
  load(params, bf, net);
  std::vector<double> g(CGKSO_MLP_NPARAM, 0.0);
  double loss = 0.0;
  for (long i = 0; i < n; ++i) {
    Acts a;
    forward_one(net, x + i * 64, bf, a);
    const double z = a.z4, yy = y[i];
    // BCE with logits: max(z,0) - y z + log(1 + exp(-|z|))
    loss += std::fmax(z, 0.0) - yy * z + std::log1p(std::exp(-std::fabs(z)));
    const double dz4 = (1.0 / (1.0 + std::exp(-z)) - yy) / static_cast<double>(n);
    double dz3[32], dz2[32], dz1[32];
    for (int j = 0; j < 32; ++j) {
      g[4192 + j] += dz4 * a.h3[j];
      dz3[j] = a.z3[j] > 0.0 ? dz4 * net.w4[j] : 0.0;
    }
    g[4224] += dz4;
    for (int j = 0; j < 32; ++j) {
      for (int k = 0; k < 32; ++k) g[3136 + j * 32 + k] += dz3[j] * a.h2[k];
      g[4160 + j] += dz3[j];
    }
    for (int k = 0; k < 32; ++k) {
      double s = 0.0;
      for (int j = 0; j < 32; ++j) s += net.W3[j][k] * dz3[j];
      dz2[k] = a.z2[k] > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < 32; ++j) {
      for (int k = 0; k < 32; ++k) g[2080 + j * 32 + k] += dz2[j] * a.h1[k];
      g[3104 + j] += dz2[j];
    }
    for (int k = 0; k < 32; ++k) {
      double s = 0.0;
      for (int j = 0; j < 32; ++j) s += net.W2[j][k] * dz2[j];
      dz1[k] = a.z1[k] > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < 32; ++j) {
      for (int k = 0; k < 64; ++k) g[j * 64 + k] += dz1[j] * a.x[k];
      g[2048 + j] += dz1[j];
    }
  }
  std::memcpy(grad, g.data(), sizeof(double) * CGKSO_MLP_NPARAM);
  return loss / static_cast<double>(n);
}

}  // extern "C"
