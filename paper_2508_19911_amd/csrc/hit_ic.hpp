// hit_ic.hpp -- host-side initial condition of decaying isotropic turbulence (arXiv 2508.19911,
// Sec. 4 test cases of compressible turbulence; the spectrum follows the common set-up
// E(k) ~ k^4 exp(-2 k^2 / k0^2)).
//
// A seeded real white-noise field per velocity component is transformed to Fourier space, shaped by
// |u_k| ~ k exp(-k^2/k0^2) for 1 <= |k| <= n/2 (integer wavenumbers of the box), projected onto
// divergence-free fields, and brought back as exact cell averages (the factor
// prod_d sin(k_d h/2)/(k_d h/2)) together with the exact cell-averaged velocity gradients.  One global
// factor then sets <|u|^2> = 3 (u_rms = 1 per component).  rho = 1, uniform p = c^2/gamma with
// c = sqrt(3)/Ma_t; the energy takes the cell-averaged velocity.
//
// Random numbers: a counter-based generator, so that any implementation reproduces the field from
// the seed alone.  The 64-bit value of counter i is the SplitMix64 output function (Steele, Lea and
// Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) applied to
// seed + (i + 1) * 0x9e3779b97f4a7c15; uniforms are (value >> 11) + 1/2 over 2^53, and normal j
// is the Box-Muller pair of uniforms 2m, 2m+1 (m = j / 2): cos for even j, sin for odd j.  Normal
// j = c N + cell feeds component c at cell (x fastest).
//
// The transforms are radix-2 complex FFTs along each axis (so n must be a power of two), with the
// sign and scaling conventions of X_k = sum_n x_n e^{-2 pi i k n / N} and its inverse with 1/N.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

namespace cgks {
namespace hit {

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
inline double uniform(uint64_t seed, uint64_t i) {
  const uint64_t v = mix64(seed + (i + 1) * 0x9e3779b97f4a7c15ULL);
  return ((double)(v >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
inline double normal(uint64_t seed, uint64_t j) {
  const uint64_t m = j >> 1;
  const double u1 = uniform(seed, 2 * m), u2 = uniform(seed, 2 * m + 1);
  const double r = std::sqrt(-2.0 * std::log(u1));
  const double th = 2.0 * M_PI * u2;
  return (j & 1) ? r * std::sin(th) : r * std::cos(th);
}

// run f(lo, hi) over [0, n) on up to 16 host threads
template <class F>
void parallel_for(long long n, F f) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const long long nt = std::min<long long>(hw, std::max<long long>(1, n / 64));
  if (nt <= 1) {
    f(0LL, n);
    return;
  }
  std::vector<std::thread> th;
  for (long long t = 0; t < nt; ++t) th.emplace_back(f, n * t / nt, n * (t + 1) / nt);
  for (auto& x : th) x.join();
}

typedef std::complex<double> cplx;

// in-place radix-2 FFT of a line of length n (a power of two), elements stride s apart; sign -1
// forward, +1 inverse (unscaled)
inline void fft_line(cplx* a, int n, long long s, int sign, const std::vector<cplx>& tw, cplx* buf) {
  for (int i = 0; i < n; ++i) buf[i] = a[i * s];
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(buf[i], buf[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1, step = n / len;
    for (int i = 0; i < n; i += len)
      for (int k = 0; k < half; ++k) {
        const cplx w = sign < 0 ? tw[k * step] : std::conj(tw[k * step]);
        const cplx u = buf[i + k], v = buf[i + k + half] * w;
        buf[i + k] = u + v;
        buf[i + k + half] = u - v;
      }
  }
  for (int i = 0; i < n; ++i) a[i * s] = buf[i];
}

// 3-D transform of an [n][n][n] array (x fastest); the inverse includes the 1/n^3
inline void fft3(std::vector<cplx>& a, int n, int sign) {
  std::vector<cplx> tw(n / 2 + 1);
  for (int k = 0; k <= n / 2; ++k) tw[k] = std::polar(1.0, -2.0 * M_PI * k / n);
  const long long n2 = (long long)n * n;
  for (int axis = 0; axis < 3; ++axis) {
    const long long s = axis == 0 ? 1 : (axis == 1 ? n : n2);
    parallel_for(n2, [&](long long lo, long long hi) {
      std::vector<cplx> buf(n);
      for (long long l = lo; l < hi; ++l) {
        const long long a0 = l / n, a1 = l % n;  // the two other indices
        long long base;
        if (axis == 0) base = a0 * n2 + a1 * n;
        else if (axis == 1) base = a0 * n2 + a1;
        else base = a0 * n + a1;
        fft_line(a.data() + base, n, s, sign, tw, buf.data());
      }
    });
  }
  if (sign > 0) {
    const double sc = 1.0 / ((double)n2 * n);
    for (auto& x : a) x *= sc;
  }
}

// q[5][N], g[15][N] of the field on an n^3 box of side L (n a power of two)
inline void field(int n, double L, double gamma, double ma_t, double k0, uint64_t seed, double* q, double* g) {
  const long long N = (long long)n * n * n;
  std::vector<int> kint(n);
  for (int i = 0; i < n; ++i) kint[i] = i <= (n - 1) / 2 ? i : i - n;  // the FFT frequency order
  const double kscale = 2.0 * M_PI / L;
  std::vector<cplx> uh[3];
  for (int c = 0; c < 3; ++c) {
    uh[c].resize(N);
    parallel_for(N, [&](long long lo, long long hi) {
      for (long long cell = lo; cell < hi; ++cell) uh[c][cell] = cplx(normal(seed, (uint64_t)(c * N + cell)), 0.0);
    });
    fft3(uh[c], n, -1);
  }
  // shape, project, cell-average factor
  parallel_for(N, [&](long long lo, long long hi) {
    for (long long cell = lo; cell < hi; ++cell) {
      const int kx = kint[cell % n], ky = kint[(cell / n) % n], kz = kint[cell / ((long long)n * n)];
      const double K2 = (double)kx * kx + (double)ky * ky + (double)kz * kz;
      const double K = std::sqrt(K2);
      double amp = 0.0;
      if (K >= 1.0 && K <= 0.5 * n) amp = K * std::exp(-(K / k0) * (K / k0));
      const double kv[3] = {(double)kx, (double)ky, (double)kz};
      cplx u[3] = {uh[0][cell] * amp, uh[1][cell] * amp, uh[2][cell] * amp};
      if (K2 > 0.0) {
        const cplx kdu = kv[0] * u[0] + kv[1] * u[1] + kv[2] * u[2];
        for (int c = 0; c < 3; ++c) u[c] -= kv[c] * kdu / K2;
      }
      double cavg = 1.0;
      for (int d = 0; d < 3; ++d) {
        const double x = M_PI * kv[d] / n;  // k_d h / 2
        cavg *= x == 0.0 ? 1.0 : std::sin(x) / x;
      }
      for (int c = 0; c < 3; ++c) uh[c][cell] = u[c] * cavg;
    }
  });
  // velocities and their derivatives (i k_d u_k)
  std::vector<double> u(3 * N), du(9 * N);
  std::vector<cplx> w(N);
  for (int c = 0; c < 3; ++c) {
    w = uh[c];
    fft3(w, n, +1);
    for (long long cell = 0; cell < N; ++cell) u[c * N + cell] = w[cell].real();
    for (int d = 0; d < 3; ++d) {
      parallel_for(N, [&](long long lo, long long hi) {
        for (long long cell = lo; cell < hi; ++cell) {
          const int kk = d == 0 ? kint[cell % n] : (d == 1 ? kint[(cell / n) % n] : kint[cell / ((long long)n * n)]);
          w[cell] = uh[c][cell] * cplx(0.0, kscale * kk);
        }
      });
      fft3(w, n, +1);
      for (long long cell = 0; cell < N; ++cell) du[(c * 3 + d) * N + cell] = w[cell].real();
    }
  }
  double s2 = 0.0;
  for (long long cell = 0; cell < N; ++cell)
    s2 += u[cell] * u[cell] + u[N + cell] * u[N + cell] + u[2 * N + cell] * u[2 * N + cell];
  const double scale = std::sqrt(3.0 / (s2 / (double)N));
  const double c_snd = std::sqrt(3.0) / ma_t;
  const double p = c_snd * c_snd / gamma;
  for (long long cell = 0; cell < N; ++cell) {
    const double ux = u[cell] * scale, uy = u[N + cell] * scale, uz = u[2 * N + cell] * scale;
    q[cell] = 1.0;
    q[N + cell] = ux;
    q[2 * N + cell] = uy;
    q[3 * N + cell] = uz;
    q[4 * N + cell] = p / (gamma - 1.0) + 0.5 * (ux * ux + uy * uy + uz * uz);
    const double uu[3] = {ux, uy, uz};
    for (int d = 0; d < 3; ++d) {
      double e = 0.0;
      g[(5 * d) * N + cell] = 0.0;
      for (int c = 0; c < 3; ++c) {
        const double dv = du[(c * 3 + d) * N + cell] * scale;
        g[(5 * d + 1 + c) * N + cell] = dv;
        e += uu[c] * dv;
      }
      g[(5 * d + 4) * N + cell] = e;
    }
  }
}

}  // namespace hit
}  // namespace cgks
