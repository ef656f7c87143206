// common.hpp -- shared device helpers for the CGKS-5th / GKS-2nd kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace cgks {

// Math in the bulk type.  FP64: the device library's correctly-rounded / few-ulp routines.  The FP32
// form uses the hardware square root, reciprocal square root and base-2 exponential (about 1 ulp;
// e^x = 2^(x log2 e) adds a relative error of about |x| 6e-8 from the rounded product).  The host
// build of the same code (tests) uses the C library throughout.
__host__ __device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__host__ __device__ __forceinline__ double dexp(double x) { return exp(x); }
__host__ __device__ __forceinline__ double dexpm1(double x) { return expm1(x); }
__host__ __device__ __forceinline__ double derfc(double x) { return erfc(x); }
__host__ __device__ __forceinline__ float dsqrt(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}
__host__ __device__ __forceinline__ float drsq(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}
__host__ __device__ __forceinline__ float dexp(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
#else
  return expf(x);
#endif
}
// e^x - 1 without cancellation near 0: the Taylor series to x^8 for |x| < 1/2 (truncation below
// 1e-8 relative), e^x - 1 elsewhere (-1 for x = -inf)
__host__ __device__ __forceinline__ float dexpm1(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  float p = 1.0f / 40320.0f;
  p = p * x + 1.0f / 5040.0f;
  p = p * x + 1.0f / 720.0f;
  p = p * x + 1.0f / 120.0f;
  p = p * x + 1.0f / 24.0f;
  p = p * x + 1.0f / 6.0f;
  p = p * x + 0.5f;
  p = p * x + 1.0f;
  p = p * x;
  const float e = dexp(x) - 1.0f;
  return fabsf(x) < 0.5f ? p : e;
#else
  return expm1f(x);
#endif
}
// 1/sqrt(x) in FP64: the hardware FP32 estimate refined by two Newton steps (relative error of a
// few 1e-16 for x in the normal FP32 range); the host build uses the C library.
__host__ __device__ __forceinline__ double rsqrt64(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  // Newton step y <- y + y (1/2 - x y^2 / 2): its constants are inline operands of the FP64 FMA
  double y = (double)__builtin_amdgcn_rsqf((float)x);
  const double mhx = -0.5 * x;
  y = fma(y, fma(mhx * y, y, 0.5), y);
  y = fma(y, fma(mhx * y, y, 0.5), y);
  return y;
#else
  return 1.0 / sqrt(x);
#endif
}

// 1/x in FP64: the hardware FP32 estimate refined by two Newton steps (error of an ulp or two for x in
// the normal FP32 range; the IEEE division costs about twice the instructions); the host build divides.
__host__ __device__ __forceinline__ double rcp64(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double y = (double)__builtin_amdgcn_rcpf((float)x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
#else
  return 1.0 / x;
#endif
}

// Coefficients of normal_split's two Maclaurin series, highest order first (Horner): erf(x) =
// (2/sqrt(pi)) x sum_n y^n / (n! (2n+1)), n = 0..11, and e^y = sum_n y^n / n!, n = 0..12, with y = -x^2.
// Kernels receive them as an argument, so they sit in scalar registers: an FP64 FMA takes no literal
// operand on this architecture, and as literals every one cost two vector moves per use.
struct SplitSeries {
  double erf_c[12];
  double exp_c[13];
};
inline SplitSeries make_split_series() {
  SplitSeries s;
  double fact = 1.0;  // n!, exact in FP64 for these n
  for (int n = 0; n <= 12; ++n) {
    if (n > 0) fact *= n;
    if (n <= 11) s.erf_c[11 - n] = 1.0 / (fact * (2 * n + 1));
    s.exp_c[12 - n] = 1.0 / fact;
  }
  return s;
}

// The split at u = 0 of a Maxwellian's normal velocity (mean U, variance var = p/rho), in FP64:
// pp = P(u > 0) = erfc(-x)/2 and pm = P(u < 0) = erfc(x)/2 with x = U/sqrt(2 var), and
// tail = e^{-x^2} sqrt(var/(2 pi)), so that <u>_{u>0} = U pp + tail and <u>_{u<0} = U pm - tail.
// For |x| < 1/2 erf(x) and e^{-x^2} are their Maclaurin series, truncated below 1e-17 (for |x| < 1/8,
// where every point of a low-Mach flow lies, the first 7 and 8 terms reach that); elsewhere the
// library's erfc and exp.  D is double (or a counting type).
template <class D>
__host__ __device__ __forceinline__ void normal_split(D U, D var, D& pp, D& pm, D& tail, const SplitSeries& ss) {
  const D isv = rsqrt64(var);
  const D x = U * isv * D(0.70710678118654752440);
  const D y = -(x * x);
  D g;
  if (fabs(x) < D(0.125)) {
    // omitted terms: (1/64)^7 / (7! 15) < 3e-18 and (1/64)^8 / 8! < 1e-19
    D s = D(ss.erf_c[5]);
#pragma unroll
    for (int k = 6; k < 12; ++k) s = s * y + D(ss.erf_c[k]);
    const D he = D(0.56418958354775628695) * x * s;  // erf(x) / 2
    pp = D(0.5) + he;
    pm = D(0.5) - he;
    g = D(ss.exp_c[5]);
#pragma unroll
    for (int k = 6; k < 13; ++k) g = g * y + D(ss.exp_c[k]);
  } else if (fabs(x) < D(0.5)) {
    D s = D(ss.erf_c[0]);
#pragma unroll
    for (int k = 1; k < 12; ++k) s = s * y + D(ss.erf_c[k]);
    const D he = D(0.56418958354775628695) * x * s;  // erf(x) / 2
    pp = D(0.5) + he;
    pm = D(0.5) - he;
    g = D(ss.exp_c[0]);
#pragma unroll
    for (int k = 1; k < 13; ++k) g = g * y + D(ss.exp_c[k]);
  } else {
    const D c = D(0.5) * derfc(fabs(x));
    if (x > D(0)) {
      pm = c;
      pp = D(1) - c;
    } else {
      pp = c;
      pm = D(1) - c;
    }
    g = dexp(y);
  }
  tail = g * (var * isv) * D(0.39894228040143267794);
}

// reciprocal in the bulk type: IEEE 1/x in FP64; the hardware reciprocal (1 ulp) in the FP32 form
__host__ __device__ __forceinline__ double drcp(double x) { return 1.0 / x; }
__host__ __device__ __forceinline__ float drcp(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

// conversion of a data value (not a constant) to the bulk type; the second argument only selects the
// overload (a counting type can supply its own)
template <class T>
__host__ __device__ __forceinline__ T data_cast(double x, T*) {
  return T(x);
}
template <class T>
__host__ __device__ __forceinline__ T data(double x) {
  return data_cast(x, static_cast<T*>(nullptr));
}

// Grid geometry and the periodic neighbour arithmetic.
struct Grid {
  int nx, ny, nz;
  long long N;
  double h[3];
  double ih[3];
};

__host__ __device__ __forceinline__ int wrap_m(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__host__ __device__ __forceinline__ int wrap_p(int i, int n) { return i == n - 1 ? 0 : i + 1; }
__host__ __device__ __forceinline__ int wrap_o(int i, int o, int n) {
  int r = i + o;
  r = r < 0 ? r + n : r;
  return r >= n ? r - n : r;
}

// Loads and stores as (uniform base pointer, 32-bit element index): the address is an SGPR pair plus
// a zero-extended 32-bit VGPR byte offset, so no 64-bit per-lane address is kept live.  Every plane
// holds fewer than 2^29 elements (checked when a context is created).
template <class T>
__host__ __device__ __forceinline__ T ld(const T* __restrict__ base, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
}
template <class T>
__host__ __device__ __forceinline__ void st(T* __restrict__ base, uint32_t idx, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(T)) = v;
}
// A streamed result: an array far larger than the caches, written once and read by a later launch.
// The non-temporal hint keeps it from allocating cache lines on the way out (measured on the
// coefficient blocks: 0.46 -> 0.36 ms per FP32 launch at 128^3, bit-identical results).
template <class T>
__host__ __device__ __forceinline__ void st_stream(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// Plane accessors for gathers.  PtrPlane reads through a pointer (host instantiations, such as the
// flop counter).  BufPlane (device) reads through a buffer resource: the plane's base and size sit
// in scalar registers and each lane supplies a 32-bit byte offset, so a gather of many planes at the
// same offsets needs no per-load address arithmetic; a read beyond the plane returns 0.
template <class T>
struct PtrPlane {
  const T* p;
  __host__ __device__ T operator()(uint32_t byte_off) const {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + byte_off);
  }
};
constexpr int BUFFER_RSRC_WORD3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)
template <class T>
struct BufPlane {
#ifdef __HIP_DEVICE_COMPILE__
  __amdgpu_buffer_rsrc_t r;
#else
  const T* p;  // the host pass only parses device code
#endif
  __device__ BufPlane(const T* base, long long n) {
#ifdef __HIP_DEVICE_COMPILE__
    // size in bytes as a 32-bit field (planes hold fewer than 2^29 elements: below 4 GiB)
    r = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0,
                                          (int)(uint32_t)(n * (long long)sizeof(T)), BUFFER_RSRC_WORD3);
#else
    p = base;
    (void)n;
#endif
  }
  __device__ T operator()(uint32_t byte_off) const {
#ifdef __HIP_DEVICE_COMPILE__
    if constexpr (sizeof(T) == 8)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0));
    else
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
#else
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + byte_off);
#endif
  }
};

// A store of element idx of a plane of n elements through a buffer resource made for the plane: the
// plane's base sits in scalar registers and the lane supplies a 32-bit byte offset, so a run of stores
// into many planes at one offset needs no per-lane 64-bit address arithmetic.
template <class T>
__device__ __forceinline__ void st_plane(T* base, long long n, uint32_t idx, T v) {
#ifdef __HIP_DEVICE_COMPILE__
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      base, (short)0, (int)(uint32_t)(n * (long long)sizeof(T)), BUFFER_RSRC_WORD3);
  if constexpr (sizeof(T) == 8) {
    using B64 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B64, v), r, (int)(idx * 8u), 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)(idx * 4u), 0, 0);
  }
#else
  base[idx] = v;
#endif
}

// Exchange inside a quad of lanes (DPP quad_perm, a VALU operand modifier; no LDS traffic):
// QUAD_XOR1 = lanes (1,0,3,2), QUAD_XOR2 = lanes (2,3,0,1).  Every lane of a quad has a source lane,
// so the moved value never falls back to the "old" operand; passing the source itself there (with
// bound_ctrl) lets the compiler fold the move into the consuming add.
constexpr int QUAD_XOR1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);
constexpr int QUAD_XOR2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);
template <int CTRL>
__device__ __forceinline__ float quad_perm(float x) {
  const int b = __builtin_bit_cast(int, x);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double quad_perm(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
  const int plo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, true);
  const int phi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)phi << 32) | (unsigned)plo);
}
// sum over the 4 lanes of a quad, in the order (x + x^1) + (x + x^1)^2
template <class T>
__device__ __forceinline__ T quad_sum(T x) {
  x += quad_perm<QUAD_XOR1>(x);
  return x + quad_perm<QUAD_XOR2>(x);
}

// XCD-aware block order.  Workgroups are handed to the 8 XCDs round robin (block b runs on XCD b mod
// 8), and each XCD has its own L2.  The remap gives every XCD a contiguous range of logical blocks, so
// neighbouring blocks (which share halo data) run on the same L2.  A bijection on [0, nb).
constexpr int NUM_XCD = 8;
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
  const unsigned q = nb / NUM_XCD, r = nb % NUM_XCD;
  const unsigned x = b % NUM_XCD, i = b / NUM_XCD;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// face-frame permutation: the face of axis d sees (normal, t1, t2) = axes (d, d+1, d+2) mod 3
__host__ __device__ constexpr int perm(int d, int k) { return (d + k) % 3; }

}  // namespace cgks
