// flopcount.hip -- algorithmic flop count of the sweep's arithmetic, by instantiating the very same
// device templates on the host with a counting scalar type.
//
// Convention: add, sub, mul, div = 1 flop; fma = 2; sqrt, exp, expm1, erfc = 1 each (reported
// separately as transcendentals).  Comparisons, min/max, abs and conversions are not counted.  The
// flux is instantiated with the counting type for both its bulk and its FP64 arithmetic; the FP64
// differences Q - Q0 of the stencil, written outside the templates, are added by hand below.
//
// Build and run (host only, no GPU needed):
//   hipcc -std=c++17 -O1 --offload-arch=gfx950 paper_2508_19911_amd/csrc/flopcount.hip -o flopcount
//   ./flopcount        -> one JSON line
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace fc {
struct Fl;
}
#include "kernels.hpp"

namespace fc {
// Expression nodes are hash-consed: an operation on the same operands is created (and counted) once,
// and operations on constants fold to constants -- the count of the formulation after common-
// subexpression elimination, which is what the compiled kernel executes at most.
long long n_flop = 0, n_trans = 0;
struct Node {
  char op;
  int a, b, c;
  double v;
};
std::vector<Node> nodes;
std::map<std::tuple<char, int, int, int, uint64_t>, int> memo;

inline bool is_const(int id) { return nodes[id].op == 'k'; }
inline int mk(char op, int a, int b, int c, double v, int cost, bool trans = false) {
  if (op == 'l') {  // an input leaf: always fresh, never constant
    nodes.push_back({op, -1, -1, -1, v});
    return (int)nodes.size() - 1;
  }
  const bool konst = (a < 0 || is_const(a)) && (b < 0 || is_const(b)) && (c < 0 || is_const(c));
  uint64_t bits = 0;
  if (konst) {
    std::memcpy(&bits, &v, 8);
    op = 'k';
    a = b = c = -1;
  } else if ((op == '+' || op == '*') && a > b) {
    std::swap(a, b);
  }
  auto key = std::make_tuple(op, a, b, c, bits);
  auto it = memo.find(key);
  if (it != memo.end()) return it->second;
  nodes.push_back({op, a, b, c, v});
  const int id = (int)nodes.size() - 1;
  memo[key] = id;
  if (!konst) {
    n_flop += cost;
    if (trans) ++n_trans;
  }
  return id;
}

struct Fl {
  int id;
  Fl() : id(mk('k', -1, -1, -1, 0.0, 0)) {}
  Fl(double x) : id(mk('k', -1, -1, -1, x, 0)) {}
  explicit operator double() const { return nodes[id].v; }
  double v() const { return nodes[id].v; }
};
inline Fl mkf(char op, Fl a, Fl b, double v, int cost = 1) {
  Fl r;
  r.id = mk(op, a.id, b.id, -1, v, cost);
  return r;
}
inline Fl operator+(Fl a, Fl b) { return mkf('+', a, b, a.v() + b.v()); }
inline Fl operator-(Fl a, Fl b) { return mkf('-', a, b, a.v() - b.v()); }
inline Fl operator*(Fl a, Fl b) { return mkf('*', a, b, a.v() * b.v()); }
inline Fl operator/(Fl a, Fl b) { return mkf('/', a, b, a.v() / b.v()); }
inline Fl operator-(Fl a) { return mkf('n', a, Fl(0.0), -a.v(), 0); }
inline Fl& operator+=(Fl& a, Fl b) { a = a + b; return a; }
inline Fl& operator-=(Fl& a, Fl b) { a = a - b; return a; }
inline Fl& operator*=(Fl& a, Fl b) { a = a * b; return a; }
inline bool operator>(Fl a, Fl b) { return a.v() > b.v(); }
inline bool operator<(Fl a, Fl b) { return a.v() < b.v(); }
inline Fl fma(Fl a, Fl b, Fl c) {
  Fl r;
  r.id = mk('f', a.id, b.id, c.id, a.v() * b.v() + c.v(), 2);
  return r;
}
inline Fl fmin(Fl a, Fl b) { return mkf('m', a, b, a.v() < b.v() ? a.v() : b.v(), 0); }
inline Fl fabs(Fl a) { return mkf('a', a, Fl(0.0), a.v() < 0 ? -a.v() : a.v(), 0); }
inline Fl un(char op, Fl x, double v) {
  Fl r;
  r.id = mk(op, x.id, -1, -1, v, 1, true);
  return r;
}
// the bulk-type math of the device code, found by argument-dependent lookup
inline Fl dsqrt(Fl x) { return un('s', x, std::sqrt(x.v())); }
inline Fl dexp(Fl x) { return un('e', x, std::exp(x.v())); }
inline Fl dexpm1(Fl x) { return un('x', x, std::expm1(x.v())); }
inline Fl derfc(Fl x) { return un('r', x, std::erfc(x.v())); }
inline Fl drcp(Fl x) { return mkf('/', Fl(1.0), x, 1.0 / x.v()); }
// FP64 reciprocal of the device: a hardware estimate (1 transcendental) and two Newton steps
inline Fl rcp64(Fl x) {
  Fl y = un('c', x, 1.0 / x.v());
  y = fma(y, fma(-x, y, Fl(1.0)), y);
  y = fma(y, fma(-x, y, Fl(1.0)), y);
  return y;
}
// FP64 reciprocal square root of the device: a hardware estimate (1 transcendental) and two Newton
// steps, written out so that their operations are counted
inline Fl rsqrt64(Fl x) {
  Fl y = un('q', x, 1.0 / std::sqrt(x.v()));
  const Fl mhx = Fl(-0.5) * x;
  y = fma(y, fma(mhx * y, y, Fl(0.5)), y);
  y = fma(y, fma(mhx * y, y, Fl(0.5)), y);
  return y;
}
inline Fl dfma(Fl a, Fl b, Fl c) { return fma(a, b, c); }
}  // namespace fc

using namespace cgks;
using fc::Fl;

// an input value: an opaque leaf (not a constant, so nothing folds through it)
static Fl leaf(double v) {
  Fl r;
  r.id = fc::mk('l', -1, -1, -1, v, 0);
  return r;
}
namespace fc {
// data values enter the counted arithmetic as leaves (found by argument-dependent lookup)
inline Fl data_cast(double x, Fl*) { return leaf(x); }
}  // namespace fc

static void reset() {
  fc::n_flop = fc::n_trans = 0;
  fc::memo.clear();
  fc::nodes.clear();
}

int main() {
  // --- k_flux5 per face: the 10 (variable, side) polynomials at the 4 Gauss points, then per point
  //     the flux (its outputs weighted by 1/4) and the 4-lane Gauss sum of its 30 outputs
  const FluxParams fp = make_flux_params(1.4, 6.25e-4, 71.43, 0.72, 0.05, 10.0);
  double WL[5] = {1.0, 0.3, 0.1, -0.2, 180.0}, WR[5] = {1.01, 0.31, 0.09, -0.21, 180.2};
  Fl DL[15], DR[15], VL[5], VR[5], out[25], Fn[5];
  Fl a[34];
  reset();
  for (int m = 0; m < 34; ++m) a[m] = leaf(1e-3 * (m + 1));
  Fl val[4], der[4][3];
  eval_face<1>(a, leaf(-1.0), val, der);
  const long long eval_face_flops = fc::n_flop;
  // per face: 10 (variable, side) polynomials, each evaluated at the 4 points, plus per point three
  // derivative scalings (Q0 + value is counted inside the flux)
  const long long state_face = 10 * (eval_face_flops + 4 * 3);
  reset();
  for (int q = 0; q < 15; ++q) {
    DL[q] = leaf(0.01 * (q + 1));
    DR[q] = leaf(0.011 * (q + 1));
  }
  for (int v = 0; v < 5; ++v) {
    VL[v] = leaf(1e-3 * (v + 1));
    VR[v] = leaf(-1e-3 * (v + 2));
  }
  gks_flux<Fl, true, Fl>(fp, 1e-3, WL, VL, DL, WR, VR, DR, Fn, out, NoPark(), 0.25);
  const long long flux_flops = fc::n_flop;
  const long long flux_trans = fc::n_trans;
  const long long reduce_flops = 30 * 2;  // two lane sums per output

  // --- one cell of k_coef: stencil data (h dQ products counted by the type, 18 FP64 differences by
  //     hand), a = R d, and optionally GENO
  const int N = 27;
  static double Qv[27];
  static Fl Gv[3 * 27];
  uint32_t oq[19], og[19];
  for (int s = 0; s < 19; ++s) {
    const uint32_t c = (tab::SOFF[s][2] + 1) * 9 + (tab::SOFF[s][1] + 1) * 3 + (tab::SOFF[s][0] + 1);
    oq[s] = c * (uint32_t)sizeof(double);
    og[s] = c * (uint32_t)sizeof(Fl);
  }
  Grid g{3, 3, 3, 27, {0.1, 0.1, 0.1}, {10, 10, 10}};
  Fl dface[6], g0[3];
  reset();
  for (int c = 0; c < N; ++c) {
    Qv[c] = 1.0 + 0.01 * c;
    for (int e = 0; e < 3; ++e) Gv[e * N + c] = leaf(0.02 * c + e);
  }
  for (int m = 0; m < 34; ++m) a[m] = Fl(0.0);
  const PtrPlane<double> qa{Qv};
  const PtrPlane<Fl> ga[3] = {{Gv}, {Gv + N}, {Gv + 2 * N}};
  gather_coefficients<Fl>(g, qa, ga, oq, og, Qv[13], a, dface, g0);
  const long long coef_var = fc::n_flop + 18;
  const long long geno_base = fc::n_flop;
  geno_blend(dface, g0, a, GenoParams{0.85, 1e-15, 0.01}, leaf(0.01));
  const long long geno_var = fc::n_flop - geno_base;

  // --- k_update5 per cell: per variable and direction L (3), Lt (3), two interface sums (3 each),
  //     then the stage-1 combination (Q*, Acc: 9 per variable; grad*: 2 per sum)
  const long long update_cell = 5 * (3 * (3 + 3 + 3 + 3) + 9) + 15 * 2;

  // one direction: the state of the low face and the flux at its 4 Gauss points
  const long long flux_launch_per_cell = state_face + 4 * (flux_flops + reduce_flops);
  const long long cell_stage_linear = 5 * coef_var + 3 * flux_launch_per_cell + update_cell;
  const long long cell_stage_geno = cell_stage_linear + 5 * geno_var;
  std::printf(
      "{\"eval_face\": %lld, \"state_per_face\": %lld, \"flux_per_gp\": %lld, \"flux_transcendentals\": %lld, "
      "\"reduce_per_gp\": %lld, \"flux_launch_per_cell\": %lld, \"coef_per_var\": %lld, \"geno_per_var\": %lld, "
      "\"update_per_cell\": %lld, \"cell_stage_linear\": %lld, \"cell_stage_geno\": %lld}\n",
      eval_face_flops, state_face, flux_flops, flux_trans, reduce_flops, flux_launch_per_cell, coef_var,
      geno_var, update_cell, cell_stage_linear, cell_stage_geno);
  return 0;
}
