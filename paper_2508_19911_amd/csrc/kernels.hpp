// kernels.hpp -- HIP kernels of the CGKS-5th / GKS-2nd stage sweep (gfx950).
//
// Per CGKS-5th stage (arXiv 2508.19911, Sec. 2-3):
//   k_coef   one thread per cell: gather the 19-cell stencil, P^4 coefficients (optionally GENO
//            blended) -> coefficient planes C[v*34+m][cell];
//   k_flux5  one thread per Gauss point of the face on the low side of each cell (one launch per
//            direction): both sides evaluated from the coefficients of the adjacent cells, the
//            gas-kinetic flux, the 2x2 Gauss average over 4 lanes -> face planes: F^n in FP64
//            Fd[dir*5+v][cell], and F_t and the two sides' interface values in T Fb[dir*25+n][cell];
//   k_update5 one thread per cell: L, dL/dt and the Gauss-theorem sums of the interface values
//            from the six faces, then the two-stage update (Sec. 3.4).
// GKS-2nd (Sec. 3.3): k_slopes2 (P^1 + Venkatakrishnan), k_flux2 (face midpoints), k_update2.
// Reductions (time step, diagnostics) are two-pass and deterministic.
#pragma once
#include "common.hpp"
#include "gks_flux.hpp"
#include "recon.hpp"

namespace cgks {

constexpr int BLK = 256;

__device__ __forceinline__ void cell_ijk(const Grid& g, int cell, int& i, int& j, int& k) {
  i = cell % g.nx;
  const int jk = cell / g.nx;
  j = jk % g.ny;
  k = jk / g.ny;
}

template <int DIR>
__device__ __forceinline__ int neighbour_m(const Grid& g, int cell, int i, int j, int k) {
  if constexpr (DIR == 0) return cell - i + wrap_m(i, g.nx);
  if constexpr (DIR == 1) return cell + (wrap_m(j, g.ny) - j) * g.nx;
  return cell + (wrap_m(k, g.nz) - k) * g.nx * g.ny;
}
template <int DIR>
__device__ __forceinline__ int neighbour_p(const Grid& g, int cell, int i, int j, int k) {
  if constexpr (DIR == 0) return cell - i + wrap_p(i, g.nx);
  if constexpr (DIR == 1) return cell + (wrap_p(j, g.ny) - j) * g.nx;
  return cell + (wrap_p(k, g.nz) - k) * g.nx * g.ny;
}

// ============================================================================ coefficient blocks
// The 34 coefficients of one variable of one cell are stored as chunks of 16 bytes (4 floats or 2
// doubles).  16 consecutive cells form a block; inside a block, chunk j of variable v of the 16
// cells is contiguous (256 bytes).  A lane reads a cell's coefficients with 16-byte loads at
// constant offsets from one address, and 16 lanes reading consecutive cells read 256 contiguous
// bytes per load.
template <class T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

template <class T>
struct CoefBlock {
  static constexpr int PER = 16 / (int)sizeof(T);              // coefficients per chunk
  static constexpr int NCH = (tab::NB + PER - 1) / PER;         // chunks per variable
  static constexpr int NBP = NCH * PER;                         // padded coefficients per variable
  static constexpr long long CHUNK_STRIDE = 16LL * PER;         // elements from chunk j to j + 1
  // element offset of chunk 0 of variable v of the cell
  __host__ __device__ static long long base(long long cell, int v) {
    return ((cell >> 4) * (5 * NCH) + v * NCH) * CHUNK_STRIDE + (cell & 15) * PER;
  }
  // elements of the whole array (whole blocks)
  __host__ __device__ static long long elements(long long N) { return ((N + 15) >> 4) * 5 * NCH * CHUNK_STRIDE; }
};

// ============================================================================ reconstruction
// a = R d for one variable of one cell, over the reflection orbits of the data columns: each orbit's
// data are loaded, combined into their sign-pattern sums D_k, and a[m] += RS[m][k] D_k (216 FMAs and
// the pattern sums instead of the 678 of R).  The face-neighbour differences and the cell's own
// normalised gradient are kept for GENO.  qa reads the variable's averages and ga[3] its gradient
// components; oq[s], og[s] are the byte offsets of stencil cell s for qa and for ga.

// stencil index of neighbour slot n (the data column of its value difference)
constexpr int stencil_of_slot(int n) {
  for (int s = 0; s < tab::NSTEN; ++s)
    if (tab::NEIGH_SLOT[s] == n) return s;
  return -1;
}

// datum of data column C: Q(neighbour) - Q0 for C < 18, else h_e dQ/dx_e of a stencil cell
template <int C, class T, class QA, class GA>
__host__ __device__ __forceinline__ T column_datum(const Grid& g, const QA& qa, const GA* ga,
                                                   const uint32_t* oq, const uint32_t* og, double q0) {
  if constexpr (C < 18) {
    constexpr int S = stencil_of_slot(C);
    static_assert(S >= 0, "neighbour slot");
    return data<T>(qa(oq[S]) - q0);
  } else {
    constexpr int S = (C - 18) / 3, E = (C - 18) % 3;
    return T(g.h[E]) * ga[E](og[S]);
  }
}

template <int K, int N, class T>
__host__ __device__ __forceinline__ T pattern_sum(const T* x) {
  T d = tab::PAT_SIGN[K][0] > 0 ? x[0] : -x[0];
  if constexpr (N > 1) d = tab::PAT_SIGN[K][1] > 0 ? d + x[1] : d - x[1];
  if constexpr (N > 2) d = tab::PAT_SIGN[K][2] > 0 ? d + x[2] : d - x[2];
  if constexpr (N > 3) d = tab::PAT_SIGN[K][3] > 0 ? d + x[3] : d - x[3];
  return d;
}

template <int K, class T, int... M>
__host__ __device__ __forceinline__ void rs_column(T d, T* a, std::integer_sequence<int, M...>) {
  ((tab::RS[M][K] != 0.0 ? (void)(a[M] = dfma(T(tab::RS[M][K]), d, a[M])) : (void)0), ...);
}

template <int O, int K, class T>
__host__ __device__ __forceinline__ void orbit_patterns(const T* x, T* a) {
  if constexpr (K < tab::ORB_PAT0[O] + tab::ORB_NPAT[O]) {
    rs_column<K>(pattern_sum<K, tab::ORB_SIZE[O]>(x), a, std::make_integer_sequence<int, tab::NB>{});
    orbit_patterns<O, K + 1>(x, a);
  }
}

// the member R of orbit O: its datum, also kept for GENO when it is a face difference or the
// cell's own gradient
template <int O, int R, class T, class QA, class GA>
__host__ __device__ __forceinline__ void orbit_member(const Grid& g, const QA& qa, const GA* ga,
                                                      const uint32_t* oq, const uint32_t* og, double q0,
                                                      T* x, T* dface, T* g0) {
  if constexpr (R < tab::ORB_SIZE[O]) {
    constexpr int C = tab::ORB_COL[O][R];
    x[R] = column_datum<C, T>(g, qa, ga, oq, og, q0);
#pragma unroll
    for (int f = 0; f < 6; ++f)
      if (C == face_slot(f)) dface[f] = x[R];
#pragma unroll
    for (int e = 0; e < 3; ++e)
      if (C == 18 + 3 * tab::CENTRE + e) g0[e] = x[R];
    orbit_member<O, R + 1>(g, qa, ga, oq, og, q0, x, dface, g0);
  }
}

template <class T, int O, class QA, class GA>
__host__ __device__ __forceinline__ void gather_orbits(const Grid& g, const QA& qa, const GA* ga,
                                                       const uint32_t* oq, const uint32_t* og, double q0,
                                                       T* a, T* dface, T* g0) {
  if constexpr (O < tab::NORB) {
    T x[4];
    orbit_member<O, 0>(g, qa, ga, oq, og, q0, x, dface, g0);
    orbit_patterns<O, tab::ORB_PAT0[O]>(x, a);
    gather_orbits<T, O + 1>(g, qa, ga, oq, og, q0, a, dface, g0);
  }
}

template <class T, class QA, class GA>
__host__ __device__ __forceinline__ void gather_coefficients(const Grid& g, const QA& qa, const GA* ga,
                                                             const uint32_t* oq, const uint32_t* og,
                                                             double q0, T* a, T* dface, T* g0) {
  gather_orbits<T, 0>(g, qa, ga, oq, og, q0, a, dface, g0);
}

// One thread per (cell, variable): blockIdx.y is the variable.  A block is a COEF_TX x COEF_TY x
// COEF_TZ tile of cells (a wave = 64 consecutive x cells).  The block first stages the variable's
// average and gradient planes over the tile and its one-cell halo in LDS, one coalesced load per
// element (the 19-point gathers straight from memory issued 76 loads per cell, most of them L1
// misses that held the vector-memory path waiting on L2); the stencil is then gathered from LDS.
constexpr int COEF_TX = 64, COEF_TY = 2, COEF_TZ = 2;
static_assert(COEF_TX * COEF_TY * COEF_TZ == BLK, "coefficient tile");
constexpr int COEF_HX = COEF_TX + 2, COEF_HY = COEF_TY + 2, COEF_HZ = COEF_TZ + 2;
constexpr int COEF_HALO = COEF_HX * COEF_HY * COEF_HZ;
__host__ __device__ inline unsigned coef_blocks(const Grid& g) {
  return (unsigned)(((g.nx + COEF_TX - 1) / COEF_TX) * ((g.ny + COEF_TY - 1) / COEF_TY) *
                    ((g.nz + COEF_TZ - 1) / COEF_TZ));
}

// x >= -1 folded into [0, n): one step for a tile inside the grid, more only for grids smaller than
// the tile
__device__ __forceinline__ int wrap_into(int x, int n) {
  if (x < 0) x += n;
  while (x >= n) x -= n;
  return x;
}

template <class T>
struct CoefShared {
  double q[COEF_HALO];     // the variable's averages over the tile and halo, x fastest
  T gr[3][COEF_HALO];      // its three gradient components
};

template <class T, int MODE>  // MODE 0 linear, 1 GENO everywhere, 2 GENO where flagged
__global__ __launch_bounds__(BLK) void k_coef(Grid g, const double* __restrict__ Q,
                                              const T* __restrict__ G,
                                              const unsigned char* __restrict__ flags,
                                              T* __restrict__ C, GenoParams gp,
                                              const double* __restrict__ ctl) {
  __shared__ CoefShared<T> sh;
  if (ctl && ctl[1] != 0.0) return;  // the step was stopped (see k_step_control)
  const int v = blockIdx.y;
  const int nby = (g.ny + COEF_TY - 1) / COEF_TY;
  // tiles run z fastest, then y, then x, and each XCD takes a contiguous range of them: a tile's
  // z-halo planes are those its predecessor just read, and its y-neighbours are nbz tiles back, all
  // through the same L2 (x fastest, the z-neighbours were 2 nbx nby tiles back: 5% slower at 256^3)
  const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int nbz = (g.nz + COEF_TZ - 1) / COEF_TZ;
  const int k0 = (b % nbz) * COEF_TZ, j0 = ((b / nbz) % nby) * COEF_TY, i0 = (b / (nbz * nby)) * COEF_TX;
  const long long N = g.N;
  const double* Qv = Q + v * N;
  const T* Gv[3] = {G + v * N, G + (5 + v) * N, G + (10 + v) * N};
  // stage the tile and its halo (periodic wrap; a tile past the grid edge wraps too)
  for (int e = threadIdx.x; e < COEF_HALO; e += BLK) {
    const int hx = e % COEF_HX, hy = (e / COEF_HX) % COEF_HY, hz = e / (COEF_HX * COEF_HY);
    const int gi = wrap_into(i0 - 1 + hx, g.nx), gj = wrap_into(j0 - 1 + hy, g.ny), gk = wrap_into(k0 - 1 + hz, g.nz);
    const uint32_t c = (uint32_t)((gk * g.ny + gj) * g.nx + gi);
    sh.q[e] = ld(Qv, c);
#pragma unroll
    for (int d = 0; d < 3; ++d) sh.gr[d][e] = ld(Gv[d], c);
  }
  __syncthreads();
  const int tx = (int)(threadIdx.x % COEF_TX), ty = (int)(threadIdx.x / COEF_TX) % COEF_TY,
            tz = (int)(threadIdx.x / (COEF_TX * COEF_TY));
  const int i = i0 + tx, j = j0 + ty, k = k0 + tz;
  if (i >= g.nx || j >= g.ny || k >= g.nz) return;
  const int cell = (k * g.ny + j) * g.nx + i;
  // byte offsets of the 19 stencil cells in the staged planes of double and of T
  uint32_t oq[tab::NSTEN], og[tab::NSTEN];
#pragma unroll
  for (int s = 0; s < tab::NSTEN; ++s) {
    const uint32_t e = (uint32_t)(((tz + 1 + tab::SOFF[s][2]) * COEF_HY + (ty + 1 + tab::SOFF[s][1])) * COEF_HX +
                                  (tx + 1 + tab::SOFF[s][0]));
    oq[s] = e * 8u;
    og[s] = e * (uint32_t)sizeof(T);
  }
  bool geno = MODE == 1;
  if constexpr (MODE == 2) geno = flags[cell] != 0;
  const PtrPlane<double> qa{sh.q};
  const PtrPlane<T> ga[3] = {PtrPlane<T>{sh.gr[0]}, PtrPlane<T>{sh.gr[1]}, PtrPlane<T>{sh.gr[2]}};
  const double q0 = sh.q[((tz + 1) * COEF_HY + (ty + 1)) * COEF_HX + (tx + 1)];
  T a[tab::NB], dface[6], g0[3];
#pragma unroll
  for (int m = 0; m < tab::NB; ++m) a[m] = T(0);
  gather_coefficients<T>(g, qa, ga, oq, og, q0, a, dface, g0);
  if (MODE != 0 && geno) {
    // the GENO floor scale of this variable needs rho and rhoE of the cell
    double q5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    q5[0] = ld(Q, (uint32_t)cell);
    q5[4] = ld(Q + 4 * N, (uint32_t)cell);
    geno_blend(dface, g0, a, gp, data<T>(gp.eps + gp.hmax2 * geno_scale(q5, v)));
  }
  using CB = CoefBlock<T>;
  using V = typename Vec16<T>::type;
  T* cb = C + CB::base(cell, v);
#pragma unroll
  for (int c = 0; c < CB::NCH; ++c) {
    V x;
#pragma unroll
    for (int e = 0; e < CB::PER; ++e) x[e] = c * CB::PER + e < tab::NB ? a[c * CB::PER + e] : T(0);
    st_stream(reinterpret_cast<V*>(cb + c * CB::CHUNK_STRIDE), x);
  }
}

// ============================================================================ CGKS-5th face flux
// One 64-lane block = the faces on the low side of 16 consecutive cells; 4 consecutive lanes hold
// the 4 Gauss points of one face.
//  1. The 10 (variable, side) polynomials of a face are split over its 4 lanes in 3 rounds; a lane
//     evaluates its polynomial at all 4 Gauss points at once (parity classes) and writes the
//     point states to LDS.
//  2. Each lane reads the two states of its own point and evaluates the gas-kinetic flux.
//  3. The 2x2 Gauss average is a 4-lane reduction; all four lanes store the face's 30 outputs.
constexpr int FLUX_FACES = 16;
constexpr int FLUX_BLK = 4 * FLUX_FACES;

template <class T>
struct FluxShared {
  T V[FLUX_FACES][4][10];        // [face][point][side * 5 + variable]: point value minus the average
  T D[FLUX_FACES][4][10][3];     // face-frame derivatives, physical units
};

// Parking place of the flux's FP64-phase values in the derivative area of FluxShared, once every lane
// has read its point's derivatives: [value][lane], so a wave's accesses are contiguous (no bank
// conflicts).  The barriers keep the stores and loads where they are written.
template <class T>
struct LdsPark {
  char* area;
  int lane;
  __device__ void save(const double* G0, const T* dS, const T* oL, const T* oR) const {
    double* d = reinterpret_cast<double*>(area);
    T* t = reinterpret_cast<T*>(area + 5 * FLUX_BLK * sizeof(double));
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      d[v * FLUX_BLK + lane] = G0[v];
      t[v * FLUX_BLK + lane] = dS[v];
      t[(5 + v) * FLUX_BLK + lane] = oL[v];
      t[(10 + v) * FLUX_BLK + lane] = oR[v];
    }
  }
  __device__ void load(double* G0, T* dS, T* oL, T* oR) const {
    const double* d = reinterpret_cast<const double*>(area);
    const T* t = reinterpret_cast<const T*>(area + 5 * FLUX_BLK * sizeof(double));
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      G0[v] = d[v * FLUX_BLK + lane];
      dS[v] = t[v * FLUX_BLK + lane];
      oL[v] = t[(5 + v) * FLUX_BLK + lane];
      oR[v] = t[(10 + v) * FLUX_BLK + lane];
    }
  }
};
static_assert(5 * FLUX_BLK * sizeof(double) + 15 * FLUX_BLK * sizeof(float) <= sizeof(FluxShared<float>::D),
              "parking area");
static_assert(5 * FLUX_BLK * sizeof(double) + 15 * FLUX_BLK * sizeof(double) <= sizeof(FluxShared<double>::D),
              "parking area");

// Occupancy: the FP32 form asks for three waves per SIMD (at most 168 VGPRs; with the FP64-phase
// values parked in LDS it needs 135 and no scratch); FP64 asks for one and keeps every value in
// registers (at two waves, 55 registers spilled and the launch took 5% longer).  A block is one wave:
// with two waves per block (32 faces, the polynomials dealt out so that one wave skips the half-idle
// third round) the barriers between the phases made the launch 12% slower.
template <class T, int DIR>
__global__ __launch_bounds__(FLUX_BLK, sizeof(T) == 8 ? 1 : 3) void k_flux5(Grid g, const double* __restrict__ Q,
                                                    const T* __restrict__ C, double* __restrict__ Fd,
                                                    T* __restrict__ Fb, FluxParams fp,
                                                    const double* __restrict__ ctl) {
  __shared__ FluxShared<T> sh;
  if (ctl[1] != 0.0) return;  // the step was stopped (see k_step_control)
  const double dt = ctl[0];
  constexpr int FP = 2 * DIR + 1;  // tables of the + face of the axis
  using CB = CoefBlock<T>;
  using V = typename Vec16<T>::type;
  const int kgp = threadIdx.x & 3;
  const int fl = threadIdx.x >> 2;
  // x faces: the low neighbour of a block's first cell lies in the previous block, so contiguous
  // block ranges per XCD keep it in the same L2.  y and z faces keep the hardware's round-robin
  // order: their neighbour blocks (nx/16 and nx ny/16 blocks back) are then on the same XCD when those
  // counts are multiples of 8, and only 1/8 as far back in its order.  (Running the y and z blocks
  // along the normal inside each XCD's range halves the z launch's reads, but the launch is ALU-bound
  // and took longer.)
  const unsigned blk = DIR == 0 ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  int cell = (int)blk * FLUX_FACES + fl;
  const bool active = cell < g.N;
  if (!active) cell = (int)g.N - 1;  // keep the lane in the reduction; its result is not stored
  int i, j, k;
  cell_ijk(g, cell, i, j, k);
  const int left = neighbour_m<DIR>(g, cell, i, j, k);
  const long long N = g.N;
  // the two cells' FP64 averages for phase 2, issued now so that their latency passes under phase 1
  double QL0[5], QR0[5];
#pragma unroll
  for (int vf = 0; vf < 5; ++vf) {
    const int vg = (vf >= 1 && vf <= 3) ? 1 + (DIR + vf - 1) % 3 : vf;
    QL0[vf] = ld(Q + vg * N, (uint32_t)left);
    QR0[vf] = ld(Q + vg * N, (uint32_t)cell);
  }
  // Phase 1.  Round r gives this lane the polynomial (side, face-frame variable) vs = 4 r + kgp; the
  // last round has 2 of them per face.  Every round's chunk loads are written ahead of the
  // evaluations, so that a round's loads are in flight while the round before is evaluated (the
  // compiler issues the last round's once the first round's registers are free).  The padding of a
  // partial last chunk is not loaded: a register whose unused part is reused by other values must
  // wait for its load, and that wait would take in every load issued before it.
  constexpr int TAIL = tab::NB - (CB::NCH - 1) * CB::PER;  // valid coefficients of the last chunk
  static_assert(TAIL == CB::PER || TAIL == 2, "last chunk: whole, or two coefficients");
  using V2 = T __attribute__((ext_vector_type(2)));
  auto chunks = [&](int r, T* x) {
    // the two lanes of a face with no polynomial in the last round load their neighbours' (and drop
    // it), so that every round's loads are unconditional and their waits exact
    const int vs = 4 * r + kgp < 10 ? 4 * r + kgp : 4 * r + kgp - 2;
    const int side = vs >= 5 ? 1 : 0;  // 0: the low cell (its + face), 1: this cell (its - face)
    const int vf = vs - 5 * side;
    const int vg = (vf >= 1 && vf <= 3) ? 1 + (DIR + vf - 1) % 3 : vf;
    const T* cb = C + CB::base(side ? cell : left, vg);
#pragma unroll
    for (int c = 0; c < CB::NCH; ++c) {
      if (c < CB::NCH - 1 || TAIL == CB::PER) {
        const V v = *reinterpret_cast<const V*>(cb + c * CB::CHUNK_STRIDE);
#pragma unroll
        for (int e = 0; e < CB::PER; ++e) x[c * CB::PER + e] = v[e];
      } else {
        const V2 v = *reinterpret_cast<const V2*>(cb + c * CB::CHUNK_STRIDE);
        x[c * CB::PER] = v[0];
        x[c * CB::PER + 1] = v[1];
      }
    }
  };
  T xs[3][tab::NB + 2];
#pragma unroll
  for (int r = 0; r < 3; ++r) chunks(r, xs[r]);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    // every lane evaluates (the wave issues the instructions either way); the two lanes of a face
    // with no polynomial in the last round do not store theirs
    const int vs = 4 * r + kgp;
    const int side = vs >= 5 ? 1 : 0;
    T val[4], der[4][3];
    eval_face<FP>(xs[r], side ? T(-1) : T(1), val, der);
    if (r < 2 || vs < 10) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        sh.V[fl][p][vs] = val[p];
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) sh.D[fl][p][vs][dd] = der[p][perm(DIR, dd)] * T(g.ih[perm(DIR, dd)]);
      }
    }
  }
  __syncthreads();
  T VL[5], VR[5], DL[15], DR[15];
#pragma unroll
  for (int vf = 0; vf < 5; ++vf) {
    VL[vf] = sh.V[fl][kgp][vf];
    VR[vf] = sh.V[fl][kgp][5 + vf];
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
      DL[dd * 5 + vf] = sh.D[fl][kgp][vf][dd];
      DR[dd * 5 + vf] = sh.D[fl][kgp][5 + vf][dd];
    }
  }
  double Fn[5];
  T out[25];
  // each point's outputs come weighted by 1/4; the 2x2 Gauss average is their sum over the face's lanes
  gks_flux<T, true>(fp, dt, QL0, VL, DL, QR0, VR, DR, Fn, out,
                    LdsPark<T>{reinterpret_cast<char*>(&sh.D[0][0][0][0]), (int)threadIdx.x}, 0.25);
#pragma unroll
  for (int n = 0; n < 5; ++n) Fn[n] = quad_sum(Fn[n]);
#pragma unroll
  for (int n = 0; n < 25; ++n) out[n] = quad_sum(out[n]);
  if (active) {
    // every lane of a face holds the face's sums; all four store them (the four lanes of a face
    // write the same bytes, which the store merges), so no lane branches on its output.  F^n goes to
    // the FP64 planes, then F_t, Q^l_n - Q0^l, Q^l_t, Q^r_n - Q0^r, Q^r_t to the T planes.
#pragma unroll
    for (int vf = 0; vf < 5; ++vf) {
      const int vg = (vf >= 1 && vf <= 3) ? 1 + perm(DIR, vf - 1) : vf;
      st_plane(Fd + (DIR * 5 + vg) * N, N, (uint32_t)cell, Fn[vf]);
#pragma unroll
      for (int blk = 0; blk < 5; ++blk)
        st_plane(Fb + (DIR * 25 + blk * 5 + vg) * N, N, (uint32_t)cell, out[blk * 5 + vf]);
    }
  }
}

// ============================================================================ sampled outputs
// out[f * n + m] = plane f at cell idx[m], for the nf planes of `planes` (element type S), as double
template <class S>
__global__ __launch_bounds__(BLK) void k_gather_cells(long long n, const uint32_t* __restrict__ idx,
                                                      const S* __restrict__ planes, int nf, long long N,
                                                      double* __restrict__ out) {
  const long long m = (long long)blockIdx.x * BLK + threadIdx.x;
  if (m >= n) return;
  const uint32_t c = idx[m];
  for (int f = 0; f < nf; ++f) out[f * n + m] = double(planes[f * N + c]);
}

// ============================================================================ unit-parity hooks
template <class T>
__global__ __launch_bounds__(64) void k_point_flux(long long n, const double* __restrict__ wl,
                                                   const double* __restrict__ wr,
                                                   double* __restrict__ out, FluxParams fp,
                                                   double dt) {
  const long long p = (long long)blockIdx.x * 64 + threadIdx.x;
  if (p >= n) return;
  double WL[5], WR[5];
  T zero[5], DL[15], DR[15];
  for (int v = 0; v < 5; ++v) {
    WL[v] = wl[p * 20 + v];
    WR[v] = wr[p * 20 + v];
    zero[v] = T(0);
  }
  for (int q = 0; q < 15; ++q) {
    DL[q] = T(wl[p * 20 + 5 + q]);
    DR[q] = T(wr[p * 20 + 5 + q]);
  }
  double Fn[5];
  T o[25];
  gks_flux<T, true>(fp, dt, WL, zero, DL, WR, zero, DR, Fn, o);
  for (int q = 0; q < 5; ++q) out[p * 30 + q] = Fn[q];
  for (int q = 0; q < 25; ++q) out[p * 30 + 5 + q] = double(o[q]);
  // interface values relative to the states given: add them back
  for (int v = 0; v < 5; ++v) {
    out[p * 30 + 10 + v] += WL[v];
    out[p * 30 + 20 + v] += WR[v];
  }
}

// ============================================================================ CGKS-5th update
struct Stage5Out {
  double* Qs;   // stage 1: Q*;           debug: dL/dt
  double* Acc;  // stage 1: Q^n + dt L + dt^2/6 L_t;  debug: L
  void* GQn;    // stage 1: sum Q_n;      debug: sum Q_n
  void* Gs;     // stage 1: grad*;        debug: sum Q_t
  double* Q;    // stage 2: Q^{n+1}
  void* G;      // stage 2: grad^{n+1}
};

template <class T, int STAGE>  // 0 debug, 1 first stage, 2 second stage
__global__ __launch_bounds__(BLK) void k_update5(Grid g, const double* __restrict__ Fd,
                                                 const T* __restrict__ Fb,
                                                 const double* __restrict__ Qn, Stage5Out o,
                                                 const double* __restrict__ ctl) {
  const int cell = blockIdx.x * BLK + threadIdx.x;
  if (cell >= g.N || ctl[1] != 0.0) return;
  const double dt = ctl[0];
  int i, j, k;
  cell_ijk(g, cell, i, j, k);
  const long long N = g.N;
  const int cp[3] = {neighbour_p<0>(g, cell, i, j, k), neighbour_p<1>(g, cell, i, j, k),
                     neighbour_p<2>(g, cell, i, j, k)};
  T* GQn = static_cast<T*>(o.GQn);
  T* Gs = static_cast<T*>(o.Gs);
  T* Gf = static_cast<T*>(o.G);
  // every load first, then every store: loads and stores complete in issue order on one counter,
  // so a load issued after a store would wait for the store
  double L[5], Lt[5], sn[3][5], st[3][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    L[v] = 0.0;
    Lt[v] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double* Fn = Fd + (long long)(d * 5) * N;
      const T* Fo = Fb + (long long)(d * 25) * N;
      L[v] -= (Fn[v * N + cp[d]] - Fn[v * N + cell]) * g.ih[d];
      Lt[v] -= (double(Fo[v * N + cp[d]]) - double(Fo[v * N + cell])) * g.ih[d];
      // this cell is the left cell of its + face and the right cell of its - face; both interface
      // values are stored relative to this cell's average, which cancels in the closed surface sum
      if constexpr (STAGE != 2)
        sn[d][v] = (double(Fo[(5 + v) * N + cp[d]]) - double(Fo[(15 + v) * N + cell])) * g.ih[d];
      st[d][v] = (double(Fo[(10 + v) * N + cp[d]]) - double(Fo[(20 + v) * N + cell])) * g.ih[d];
    }
  }
  double q[5];
  if constexpr (STAGE == 1) {
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = Qn[v * N + cell];
  } else if constexpr (STAGE == 2) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      q[v] = o.Acc[v * N + cell];
#pragma unroll
      for (int d = 0; d < 3; ++d) sn[d][v] = double(GQn[(d * 5 + v) * N + cell]);
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const long long gi = (d * 5 + v) * N + cell;
      if constexpr (STAGE == 0) {
        GQn[gi] = T(sn[d][v]);
        Gs[gi] = T(st[d][v]);
      } else if constexpr (STAGE == 1) {
        st_stream(&GQn[gi], T(sn[d][v]));
        st_stream(&Gs[gi], T(sn[d][v] + 0.5 * dt * st[d][v]));
      } else {
        st_stream(&Gf[gi], T(sn[d][v] + dt * st[d][v]));
      }
    }
    const long long qi = v * N + cell;
    if constexpr (STAGE == 0) {
      o.Acc[qi] = L[v];
      o.Qs[qi] = Lt[v];
    } else if constexpr (STAGE == 1) {
      st_stream(&o.Qs[qi], q[v] + 0.5 * dt * L[v] + 0.125 * dt * dt * Lt[v]);
      st_stream(&o.Acc[qi], q[v] + dt * L[v] + dt * dt / 6.0 * Lt[v]);
    } else {
      st_stream(&o.Q[qi], q[v] + dt * dt / 3.0 * Lt[v]);
    }
  }
}

// ============================================================================ GKS-2nd
template <class T, int LIM>
__global__ __launch_bounds__(BLK) void k_slopes2(Grid g, const double* __restrict__ Q,
                                                 T* __restrict__ S, double vk_eps2,
                                                 const double* __restrict__ ctl) {
  const int cell = blockIdx.x * BLK + threadIdx.x;
  if (cell >= g.N || (ctl && ctl[1] != 0.0)) return;  // ctl: a stopped step skips the slopes
  int i, j, k;
  cell_ijk(g, cell, i, j, k);
  const long long N = g.N;
  const int nb[6] = {neighbour_m<0>(g, cell, i, j, k), neighbour_p<0>(g, cell, i, j, k),
                     neighbour_m<1>(g, cell, i, j, k), neighbour_p<1>(g, cell, i, j, k),
                     neighbour_m<2>(g, cell, i, j, k), neighbour_p<2>(g, cell, i, j, k)};
  // all loads before the first store (loads and stores complete in issue order on one counter)
  double qc[5], qn[5][6];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    qc[v] = Q[v * N + cell];
#pragma unroll
    for (int m = 0; m < 6; ++m) qn[v][m] = Q[v * N + nb[m]];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double q0 = qc[v];
    const double* q = qn[v];
    double b[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) b[e] = 0.5 * (q[2 * e + 1] - q[2 * e]);
    double phi = 1.0;
    if constexpr (LIM) {
      double qmax = q0, qmin = q0;
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        qmax = fmax(qmax, q[m]);
        qmin = fmin(qmin, q[m]);
      }
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const double d2 = ((f % 2) ? 0.5 : -0.5) * b[f / 2];
        double pf = 1.0;
        if (d2 != 0.0) {
          const double d1 = d2 > 0.0 ? qmax - q0 : qmin - q0;
          pf = ((d1 * d1 + vk_eps2) + 2.0 * d1 * d2) / (d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + vk_eps2);
        }
        phi = fmin(phi, pf);
      }
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) st_stream(&S[(v * 3 + e) * N + cell], T(phi * b[e]));
  }
}

template <class T, int DIR>
__global__ __launch_bounds__(BLK) void k_flux2(Grid g, const double* __restrict__ Q,
                                               const T* __restrict__ S, double* __restrict__ Fd,
                                               T* __restrict__ Fb, FluxParams fp,
                                               const double* __restrict__ ctl) {
  const int cell = blockIdx.x * BLK + threadIdx.x;
  if (cell >= g.N || ctl[1] != 0.0) return;
  const double dt = ctl[0];
  int i, j, k;
  cell_ijk(g, cell, i, j, k);
  const int left = neighbour_m<DIR>(g, cell, i, j, k);
  const long long N = g.N;
  double QL[5], QR[5];
  T VL[5], VR[5], DL[15], DR[15];
#pragma unroll
  for (int vf = 0; vf < 5; ++vf) {
    const int vg = (vf >= 1 && vf <= 3) ? 1 + perm(DIR, vf - 1) : vf;
    const T* Sv = S + (long long)(vg * 3) * N;
    QL[vf] = Q[vg * N + left];
    QR[vf] = Q[vg * N + cell];
    VL[vf] = T(0.5) * Sv[DIR * N + left];
    VR[vf] = T(-0.5) * Sv[DIR * N + cell];
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
      const int e = perm(DIR, dd);
      DL[dd * 5 + vf] = Sv[e * N + left] * T(g.ih[e]);
      DR[dd * 5 + vf] = Sv[e * N + cell] * T(g.ih[e]);
    }
  }
  double Fn[5];
  T out[5];
  gks_flux<T, false>(fp, dt, QL, VL, DL, QR, VR, DR, Fn, out);
#pragma unroll
  for (int vf = 0; vf < 5; ++vf) {
    const int vg = (vf >= 1 && vf <= 3) ? 1 + perm(DIR, vf - 1) : vf;
    Fd[(DIR * 5 + vg) * N + cell] = Fn[vf];
    Fb[(DIR * 5 + vg) * N + cell] = out[vf];
  }
}

template <class T, int DEBUG>
__global__ __launch_bounds__(BLK) void k_update2(Grid g, const double* __restrict__ Fd,
                                                 const T* __restrict__ Fb, double* Q,
                                                 double* Lout, double* Ltout, const double* __restrict__ ctl) {
  const int cell = blockIdx.x * BLK + threadIdx.x;
  if (cell >= g.N || ctl[1] != 0.0) return;
  const double dt = ctl[0];
  int i, j, k;
  cell_ijk(g, cell, i, j, k);
  const long long N = g.N;
  const int cp[3] = {neighbour_p<0>(g, cell, i, j, k), neighbour_p<1>(g, cell, i, j, k),
                     neighbour_p<2>(g, cell, i, j, k)};
  // all loads before the first store (loads and stores complete in issue order on one counter)
  double L[5], Lt[5], q[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    L[v] = 0.0;
    Lt[v] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double* Fn = Fd + (long long)(d * 5) * N;
      const T* Ft = Fb + (long long)(d * 5) * N;
      L[v] -= (Fn[v * N + cp[d]] - Fn[v * N + cell]) * g.ih[d];
      Lt[v] -= (double(Ft[v * N + cp[d]]) - double(Ft[v * N + cell])) * g.ih[d];
    }
    if constexpr (!DEBUG) q[v] = Q[v * N + cell];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    if constexpr (DEBUG) {
      Lout[v * N + cell] = L[v];
      Ltout[v * N + cell] = Lt[v];
    } else {
      st_stream(&Q[v * N + cell], q[v] + (dt * L[v] + 0.5 * dt * dt * Lt[v]));
    }
  }
}

// ============================================================================ reductions
// Reduction of NV values over a block: first over the 64 lanes of each wave by cross-lane exchanges in
// a fixed butterfly (lane i combines with lane i ^ 32, ^ 16, ..., ^ 1; the operations are commutative,
// so every lane ends with the same bits), then over the block's waves through LDS, in wave order.  The
// order is the same on every run: the reductions are deterministic.
constexpr int WAVES = BLK / 64;
template <int NV, class Op>
__device__ __forceinline__ void block_reduce(double (*sh)[WAVES], double* val, Op op) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < NV; ++q) val[q] = op(q, val[q], __shfl_xor(val[q], off, 64));
  const int w = (int)(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q][w] = val[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double r = sh[q][0];
#pragma unroll
    for (int k = 1; k < WAVES; ++k) r = op(q, r, sh[q][k]);
    val[q] = r;
  }
}

struct DtOp {
  __device__ double operator()(int q, double a, double b) const {
    return q == 0 ? fmin(a, b) : fmax(a, b);
  }
};

// per block: min_i min_d h_d/(|U_d|+c), max nu, any non-physical cell, over the cells
// blockIdx.x * BLK + threadIdx.x + m gridDim.x BLK (one cell per thread when the grid covers N)
__global__ __launch_bounds__(BLK) void k_dt(Grid g, const double* __restrict__ Q, FluxParams fp,
                                            double* part) {
  __shared__ double sh[3][WAVES];
  double val[3] = {INFINITY, 0.0, 0.0};
  const long long N = g.N;
  for (long long cell = (long long)blockIdx.x * BLK + threadIdx.x; cell < N; cell += (long long)gridDim.x * BLK) {
    const double rho = Q[cell], mx = Q[N + cell], my = Q[2 * N + cell], mz = Q[3 * N + cell],
                 E = Q[4 * N + cell];
    const double U = mx / rho, V = my / rho, W = mz / rho;
    const double p = (fp.gamma - 1.0) * (E - 0.5 * rho * (U * U + V * V + W * W));
    const bool ok = rho > 0.0 && p > 0.0 && isfinite(p) && isfinite(U) && isfinite(V) && isfinite(W);
    if (ok) {
      const double c = sqrt(fp.gamma * p / rho);
      val[0] = fmin(val[0], fmin(g.h[0] / (fabs(U) + c), fmin(g.h[1] / (fabs(V) + c), g.h[2] / (fabs(W) + c))));
      if (fp.mu0 > 0.0) val[1] = fmax(val[1], viscosity<double>(fp, p / rho) / rho);
    } else {
      val[2] = 1.0;
    }
  }
  block_reduce<3>(sh, val, DtOp{});
  if (threadIdx.x == 0) {
    part[blockIdx.x * 3 + 0] = val[0];
    part[blockIdx.x * 3 + 1] = val[1];
    part[blockIdx.x * 3 + 2] = val[2];
  }
}

__global__ __launch_bounds__(BLK) void k_dt_final(int nblk, const double* __restrict__ part,
                                                  double* out) {
  __shared__ double sh[3][WAVES];
  double val[3] = {INFINITY, 0.0, 0.0};
  // unrolled so that several iterations' loads are in flight at once (one partial per block of the
  // first pass: 65 536 of them at 256^3)
#pragma unroll 8
  for (int b = threadIdx.x; b < nblk; b += BLK) {
    val[0] = fmin(val[0], part[b * 3 + 0]);
    val[1] = fmax(val[1], part[b * 3 + 1]);
    val[2] = fmax(val[2], part[b * 3 + 2]);
  }
  block_reduce<3>(sh, val, DtOp{});
  if (threadIdx.x == 0) {
    out[0] = val[0];
    out[1] = val[1];
    out[2] = val[2];
  }
}

struct DiagOp {
  __device__ double operator()(int q, double a, double b) const {
    return (q == 9 || q == 10) ? fmin(a, b) : a + b;
  }
};

// ============================================================================ step control on the device
// ctl[0] = dt of the current step, ctl[1] = 0 go / 1 stopped at t_stop / 2 stopped non-physical,
// ctl[2] = t, ctl[3] = steps done.  The stage kernels read dt from ctl and do nothing once ctl[1] is
// set, so a batch of steps runs without the host reading dt back after every step, and a stopped
// batch leaves the state of the step it stopped at.
__global__ void k_ctl_init(double* ctl, double t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl[0] = 0.0;
    ctl[1] = 0.0;
    ctl[2] = t;
    ctl[3] = 0.0;
    ctl[4] = 0.0;
  }
}
__global__ void k_ctl_set_dt(double* ctl, double dt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl[0] = dt;
    ctl[1] = 0.0;
  }
}
// lim = (min h/(|U|+c), max nu, non-physical flag) from k_dt_final; dt = CFL lim0, and
// CFL h_min^2/(3 lim1) when viscous; the last step is shortened to end at t_stop (> 0).
// ctl = (dt, stop: 1 at t_stop, 2 non-physical, t, steps taken, dt before the shortening)
__global__ void k_step_control(const double* __restrict__ lim, double* ctl, double cfl, double hmin,
                               int viscous, double t_stop) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || ctl[1] != 0.0) return;
  const double t = ctl[2];
  if (t_stop > 0.0 && t >= t_stop) {
    ctl[1] = 1.0;
    return;
  }
  if (lim[2] != 0.0) {
    ctl[1] = 2.0;
    return;
  }
  double dt = cfl * lim[0];
  if (viscous) dt = fmin(dt, cfl * hmin * hmin / (3.0 * lim[1]));
  ctl[4] = dt;
  if (t_stop > 0.0 && t + dt > t_stop) dt = t_stop - t;
  ctl[0] = dt;
}
// dt[0] = the time step of the limits lim (as k_step_control, without a t_stop), dt[1] = the
// non-physical flag of the reduction
__global__ void k_dt_value(const double* __restrict__ lim, double cfl, double hmin, int viscous, double* dt) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double d = cfl * lim[0];
  if (viscous) d = fmin(d, cfl * hmin * hmin / (3.0 * lim[1]));
  dt[0] = d;
  dt[1] = lim[2];
}
__global__ void k_step_advance(double* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && ctl[1] == 0.0) {
    ctl[2] += ctl[0];
    ctl[3] += 1.0;
  }
}

// diagnostics partials: 0 ek, 1 es, 2 ed, 3..7 sum Q, 8 flagged, 9 rho min, 10 p min
template <class T, int CENTRAL>
__global__ __launch_bounds__(BLK) void k_diag(Grid g, const double* __restrict__ Q,
                                              const T* __restrict__ G,
                                              const unsigned char* __restrict__ flags,
                                              FluxParams fp, double vol, double* part) {
  __shared__ double sh[11][WAVES];
  const int cell = blockIdx.x * BLK + threadIdx.x;
  double val[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, INFINITY, INFINITY};
  if (cell < g.N) {
    const long long N = g.N;
    double q[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = Q[v * N + cell];
    const double rho = q[0];
    const double U[3] = {q[1] / rho, q[2] / rho, q[3] / rho};
    const double p = (fp.gamma - 1.0) * (q[4] - 0.5 * rho * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
    double gr[3][4];  // d(rho, m_x, m_y, m_z)/dx_d
    if constexpr (CENTRAL) {
      int i, j, k;
      cell_ijk(g, cell, i, j, k);
      const int mp[3][2] = {{neighbour_m<0>(g, cell, i, j, k), neighbour_p<0>(g, cell, i, j, k)},
                            {neighbour_m<1>(g, cell, i, j, k), neighbour_p<1>(g, cell, i, j, k)},
                            {neighbour_m<2>(g, cell, i, j, k), neighbour_p<2>(g, cell, i, j, k)}};
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          gr[d][v] = (Q[v * N + mp[d][1]] - Q[v * N + mp[d][0]]) / (2.0 * g.h[d]);
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = 0; v < 4; ++v) gr[d][v] = double(G[(d * 5 + v) * N + cell]);
    }
    double du[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int a = 0; a < 3; ++a) du[a][d] = (gr[d][1 + a] - U[a] * gr[d][0]) / rho;
    const double wx = du[2][1] - du[1][2], wy = du[0][2] - du[2][0], wz = du[1][0] - du[0][1];
    const double div = du[0][0] + du[1][1] + du[2][2];
    const double mu = viscosity<double>(fp, p / rho);
    val[0] = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / rho;
    val[1] = mu * (wx * wx + wy * wy + wz * wz);
    val[2] = mu * div * div;
#pragma unroll
    for (int v = 0; v < 5; ++v) val[3 + v] = q[v] * vol;
    val[8] = flags ? double(flags[cell] != 0) : 1.0;
    val[9] = rho;
    val[10] = p;
  }
  block_reduce<11>(sh, val, DiagOp{});
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 11; ++q) part[blockIdx.x * 11 + q] = val[q];
}

__global__ __launch_bounds__(BLK) void k_diag_final(int nblk, const double* __restrict__ part,
                                                    double* out) {
  __shared__ double sh[11][WAVES];
  double val[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, INFINITY, INFINITY};
  for (int b = threadIdx.x; b < nblk; b += BLK)
#pragma unroll
    for (int q = 0; q < 11; ++q) val[q] = DiagOp{}(q, val[q], part[b * 11 + q]);
  block_reduce<11>(sh, val, DiagOp{});
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 11; ++q) out[q] = val[q];
}

// ============================================================================ quadrature diagnostics
// E_k, eps_S and eps_D integrated over each cell with the 3x3x3 Gauss-Legendre rule applied to the
// cell's reconstruction (Sec. 4.1, 4.2: the derivatives at the quadrature points come from the
// reconstruction): the P^4 coefficients of CGKS-5th (GENO folded in as in the scheme), or the
// limited P^1 of GKS-2nd.  At each point: rho, m, rhoE and the gradients of rho and m give
// (1/2) rho |U|^2, mu |curl U|^2 and mu (div U)^2, mu from the point's temperature.  Partials use
// the 11-slot layout of k_diag (slots 0-2; the others hold the identities) for k_diag_final.
__device__ __forceinline__ void quad_point(const FluxParams& fp, double w, const double q[5],
                                           const double (*gr)[3], double* acc) {
  const double rho = q[0];
  const double ir = 1.0 / rho;
  const double U[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
  const double p = (fp.gamma - 1.0) * (q[4] - 0.5 * rho * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
  double du[3][3];  // du[a][d] = d U_a / d x_d
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d) du[a][d] = (gr[1 + a][d] - U[a] * gr[0][d]) * ir;
  const double wx = du[2][1] - du[1][2], wy = du[0][2] - du[2][0], wz = du[1][0] - du[0][1];
  const double div = du[0][0] + du[1][1] + du[2][2];
  const double mu = viscosity<double>(fp, p * ir);
  acc[0] += w * 0.5 * rho * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
  acc[1] += w * mu * (wx * wx + wy * wy + wz * wz);
  acc[2] += w * mu * div * div;
}

__device__ __forceinline__ void quad_partials(double* part, double* acc) {
  __shared__ double sh[11][WAVES];
  double val[11] = {acc[0], acc[1], acc[2], 0, 0, 0, 0, 0, 0, INFINITY, INFINITY};
  block_reduce<11>(sh, val, DiagOp{});
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 11; ++q) part[blockIdx.x * 11 + q] = val[q];
}

// CGKS-5th: C holds the coefficient blocks of the current state.  The nine (y, z) point pairs are
// looped over; the three x points of a pair share one load of each variable's coefficients.
template <class T>
__global__ __launch_bounds__(BLK) void k_diag_quad5(Grid g, const double* __restrict__ Q,
                                                    const T* __restrict__ C, FluxParams fp,
                                                    double* part) {
  using CB = CoefBlock<T>;
  using V = typename Vec16<T>::type;
  const int cell = blockIdx.x * BLK + threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  if (cell < g.N) {
    const long long N = g.N;
    double q0[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) q0[v] = Q[v * N + cell];
#pragma unroll 1
    for (int s = 0; s < 9; ++s) {
      double qv[3][5], gr[3][4][3];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const T* cb = C + CB::base(cell, v);
        T a[CB::NBP];
#pragma unroll
        for (int c = 0; c < CB::NCH; ++c) {
          const V x = *reinterpret_cast<const V*>(cb + c * CB::CHUNK_STRIDE);
#pragma unroll
          for (int e = 0; e < CB::PER; ++e) a[c * CB::PER + e] = x[e];
        }
#pragma unroll
        for (int ix = 0; ix < 3; ++ix) {
          const int qp = 3 * s + ix;
          T val = T(0);
#pragma unroll
          for (int m = 0; m < tab::NB; ++m) val += a[m] * T(tab::PVQ[qp][m]);
          qv[ix][v] = q0[v] + double(val);
          if (v < 4) {
#pragma unroll
            for (int e = 0; e < 3; ++e) {
              T d = T(0);
#pragma unroll
              for (int m = 0; m < tab::NB; ++m)
                if (tab::BD[m][e] > 0) d += a[m] * T(tab::PDQ[qp][e][m]);
              gr[ix][v][e] = double(d) * g.ih[e];
            }
          }
        }
      }
#pragma unroll
      for (int ix = 0; ix < 3; ++ix) quad_point(fp, tab::VQ_W[3 * s + ix], qv[ix], gr[ix], acc);
    }
  }
  quad_partials(part, acc);
}

// GKS-2nd: S[(v * 3 + e) * N + cell] = the limited slope of variable v along axis e per unit of the
// normalised coordinate; the gradient is constant over the cell.
template <class T>
__global__ __launch_bounds__(BLK) void k_diag_quad2(Grid g, const double* __restrict__ Q,
                                                    const T* __restrict__ S, FluxParams fp,
                                                    double* part) {
  const int cell = blockIdx.x * BLK + threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  if (cell < g.N) {
    const long long N = g.N;
    double q0[5], sl[5][3], gr[4][3];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      q0[v] = Q[v * N + cell];
#pragma unroll
      for (int e = 0; e < 3; ++e) sl[v][e] = double(S[(v * 3 + e) * N + cell]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int e = 0; e < 3; ++e) gr[v][e] = sl[v][e] * g.ih[e];
#pragma unroll 1
    for (int qp = 0; qp < tab::NVQ; ++qp) {
      double q[5];
#pragma unroll
      for (int v = 0; v < 5; ++v)
        q[v] = q0[v] + sl[v][0] * tab::VQ_X[qp][0] + sl[v][1] * tab::VQ_X[qp][1] + sl[v][2] * tab::VQ_X[qp][2];
      quad_point(fp, tab::VQ_W[qp], q, gr, acc);
    }
  }
  quad_partials(part, acc);
}

// ============================================================================ conversions
template <class T>
__global__ __launch_bounds__(BLK) void k_convert(long long n, const double* __restrict__ src,
                                                 T* __restrict__ dst) {
  const long long idx = (long long)blockIdx.x * BLK + threadIdx.x;
  if (idx < n) dst[idx] = T(src[idx]);
}

// ============================================================================ initial conditions
struct ICParams {
  int kind;  // 0 vortex, 1 TGV, 2 supersonic TGV
  double gamma;
  double a0, a1, a2;  // vortex: strength; TGV: Ma, rho0, u0
};

__device__ __forceinline__ void ic_point(const ICParams& ip, const Grid& g, double x, double y,
                                         double z, double* c) {
  const double gm = ip.gamma;
  double rho, u, v, w, p;
  if (ip.kind == 0) {
    const double Lx = g.h[0] * g.nx, Ly = g.h[1] * g.ny;
    double dx = x - 0.5 * Lx, dy = y - 0.5 * Ly;
    dx = dx - Lx * floor(dx / Lx + 0.5);
    dy = dy - Ly * floor(dy / Ly + 0.5);
    const double r2 = dx * dx + dy * dy;
    const double f = ip.a0 / (2.0 * M_PI) * exp(0.5 * (1.0 - r2));
    u = 1.0 - f * dy;
    v = 1.0 + f * dx;
    w = 0.0;
    const double T = 1.0 - (gm - 1.0) * ip.a0 * ip.a0 / (8.0 * gm * M_PI * M_PI) * exp(1.0 - r2);
    rho = pow(T, 1.0 / (gm - 1.0));
    p = rho * T;
  } else {
    double rho0, u0, p0, amp;
    if (ip.kind == 1) {
      rho0 = ip.a1;
      u0 = ip.a2;
      p0 = rho0 * u0 * u0 / (gm * ip.a0 * ip.a0);
      amp = gm * ip.a0 * ip.a0 / 16.0;
    } else {
      rho0 = 1.0;
      p0 = 1.0;
      u0 = sqrt(gm) * ip.a0;
      amp = 1.0 / 16.0;
    }
    const double s = (cos(2.0 * x) + cos(2.0 * y)) * (cos(2.0 * z) + 2.0);
    rho = rho0 * (1.0 + amp * s);
    p = p0 * (1.0 + amp * s);
    u = u0 * sin(x) * cos(y) * cos(z);
    v = -u0 * cos(x) * sin(y) * cos(z);
    w = 0.0;
  }
  c[0] = rho;
  c[1] = rho * u;
  c[2] = rho * v;
  c[3] = rho * w;
  c[4] = p / (gm - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
}

template <class T>
__global__ __launch_bounds__(BLK) void k_ic(Grid g, ICParams ip, double* __restrict__ Q,
                                            T* __restrict__ G) {
  const int cell = blockIdx.x * BLK + threadIdx.x;
  if (cell >= g.N) return;
  int i, j, k;
  cell_ijk(g, cell, i, j, k);
  const long long N = g.N;
  // 4-point Gauss-Legendre on [-1/2, 1/2]
  const double xg[4] = {-0.43056815579702629, -0.16999052179242813, 0.16999052179242813,
                        0.43056815579702629};
  const double wg[4] = {0.17392742256872693, 0.32607257743127307, 0.32607257743127307,
                        0.17392742256872693};
  const double c0[3] = {(i + 0.5) * g.h[0], (j + 0.5) * g.h[1], (k + 0.5) * g.h[2]};
  double avg[5] = {0, 0, 0, 0, 0};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int c = 0; c < 4; ++c) {
        double s[5];
        ic_point(ip, g, c0[0] + g.h[0] * xg[c], c0[1] + g.h[1] * xg[b], c0[2] + g.h[2] * xg[a], s);
        const double wt = wg[a] * wg[b] * wg[c];
        for (int v = 0; v < 5; ++v) avg[v] += wt * s[v];
      }
  for (int v = 0; v < 5; ++v) Q[v * N + cell] = avg[v];
  for (int d = 0; d < 3; ++d) {
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    double diff[5] = {0, 0, 0, 0, 0};
    for (int sg = -1; sg <= 1; sg += 2)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          double x[3];
          x[d] = c0[d] + 0.5 * sg * g.h[d];
          x[t1] = c0[t1] + g.h[t1] * xg[a];
          x[t2] = c0[t2] + g.h[t2] * xg[b];
          double s[5];
          ic_point(ip, g, x[0], x[1], x[2], s);
          for (int v = 0; v < 5; ++v) diff[v] += sg * wg[a] * wg[b] * s[v];
        }
    for (int v = 0; v < 5; ++v) G[(d * 5 + v) * N + cell] = T(diff[v] / g.h[d]);
  }
}

}  // namespace cgks
