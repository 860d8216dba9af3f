// opcount.cpp -- the oracle's arithmetic, counted.
//
// TEST AND MEASUREMENT INFRASTRUCTURE ONLY, like the oracle itself.  This
// file compiles mfm_oracle.c unchanged except that every `double` becomes
// `Counted`, a number type that holds one double (same size and layout) and
// counts each floating-point operation done on it: additions and
// subtractions, multiplications, divisions, square roots, and powers (pow,
// exp, log).  Comparisons, fabs, fmin, fmax and floor are not counted.  The
// counts are the algorithmic work of the method as the oracle performs it,
// operation by operation: the flux loop's count per face is the one the
// benchmark's roofline divides by the kernel time.
//
// The candidate scans of the oracle (its ORC_SEARCH_BEGIN / END hooks) are
// counted apart from the loops that call them.  The build is serial (no
// OpenMP), so the counters are plain globals.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

namespace opc {
enum { ADD = 0, MUL, DIV, SQRT, POW, NKIND };
int64_t counts[2][NKIND];  // [0] the loop itself, [1] candidate scans
int phase = 0;
inline void tick(int k) { ++counts[phase][k]; }
}  // namespace opc

struct Counted {
  double v;
  Counted() = default;
  Counted(double x) : v(x) {}  // NOLINT: implicit, as a double literal would convert
  explicit operator double() const { return v; }
  explicit operator int() const { return (int)v; }
  Counted &operator+=(Counted o) { opc::tick(opc::ADD); v += o.v; return *this; }
  Counted &operator-=(Counted o) { opc::tick(opc::ADD); v -= o.v; return *this; }
  Counted &operator*=(Counted o) { opc::tick(opc::MUL); v *= o.v; return *this; }
  Counted &operator/=(Counted o) { opc::tick(opc::DIV); v /= o.v; return *this; }
};
static_assert(sizeof(Counted) == sizeof(double), "Counted must have the layout of a double");

inline Counted operator+(Counted a, Counted b) { opc::tick(opc::ADD); return a.v + b.v; }
inline Counted operator-(Counted a, Counted b) { opc::tick(opc::ADD); return a.v - b.v; }
inline Counted operator*(Counted a, Counted b) { opc::tick(opc::MUL); return a.v * b.v; }
inline Counted operator/(Counted a, Counted b) { opc::tick(opc::DIV); return a.v / b.v; }
inline Counted operator-(Counted a) { return -a.v; }
inline bool operator<(Counted a, Counted b) { return a.v < b.v; }
inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
inline bool operator<=(Counted a, Counted b) { return a.v <= b.v; }
inline bool operator>=(Counted a, Counted b) { return a.v >= b.v; }
inline bool operator==(Counted a, Counted b) { return a.v == b.v; }
inline bool operator!=(Counted a, Counted b) { return a.v != b.v; }
inline Counted sqrt(Counted a) { opc::tick(opc::SQRT); return std::sqrt(a.v); }
inline Counted pow(Counted a, Counted b) { opc::tick(opc::POW); return std::pow(a.v, b.v); }
inline Counted exp(Counted a) { opc::tick(opc::POW); return std::exp(a.v); }
inline Counted log(Counted a) { opc::tick(opc::POW); return std::log(a.v); }
inline Counted fabs(Counted a) { return std::fabs(a.v); }
inline Counted fmin(Counted a, Counted b) { return std::fmin(a.v, b.v); }
inline Counted fmax(Counted a, Counted b) { return std::fmax(a.v, b.v); }
inline Counted floor(Counted a) { return std::floor(a.v); }
inline bool isfinite(Counted a) { return std::isfinite(a.v); }

#define ORC_SEARCH_BEGIN() int opc_saved_phase_ = opc::phase; opc::phase = 1
#define ORC_SEARCH_END() opc::phase = opc_saved_phase_
#define double Counted
#include "mfm_oracle.c"
#undef double

namespace {
void reset() {
  memset(opc::counts, 0, sizeof(opc::counts));
  opc::phase = 0;
}
void report(int64_t *out) {
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < opc::NKIND; ++k) out[p * opc::NKIND + k] = opc::counts[p][k];
}
}  // namespace

// Each entry point runs the oracle function of the same name on plain double
// arrays (Counted has the layout of a double) and writes 10 counts: for the
// loop itself, then for its candidate scans, the additions, multiplications,
// divisions, square roots and powers.
extern "C" __attribute__((visibility("default"))) int opc_face(
    const orc_params *p, int64_t n, int64_t i, int64_t j, const Counted *x, const Counted *y,
    const Counted *z, const Counted *H, const Counted *V, const Counted *rho, const Counted *vx,
    const Counted *vy, const Counted *vz, const Counted *P, const Counted *B, const Counted *grad,
    double dt, Counted *c, orc_counters *cnt, int64_t *counts) {
  reset();
  int rc = orc_face(p, n, i, j, x, y, z, H, V, rho, vx, vy, vz, P, B, grad, Counted(dt), c, cnt);
  report(counts);
  return rc;
}

extern "C" __attribute__((visibility("default"))) int opc_density(
    const orc_params *p, int64_t n, const Counted *x, const Counted *y, const Counted *z,
    Counted *H, Counted *V, Counted *ncond, Counted *nngb, orc_counters *cnt, int64_t *counts) {
  reset();
  int rc = orc_density(p, n, x, y, z, H, V, ncond, nngb, cnt);
  report(counts);
  return rc;
}

extern "C" __attribute__((visibility("default"))) int opc_gradients(
    const orc_params *p, int64_t n, const Counted *x, const Counted *y, const Counted *z,
    const Counted *H, const Counted *V, const Counted *m, const Counted *vx, const Counted *vy,
    const Counted *vz, const Counted *U, Counted *rho, Counted *P, Counted *c, Counted *B,
    Counted *grad, Counted *alpha, Counted *ncond, Counted *dt_i, orc_counters *cnt,
    int64_t *counts) {
  reset();
  int rc = orc_gradients(p, n, x, y, z, H, V, m, vx, vy, vz, U, rho, P, c, B, grad, alpha, ncond,
                         dt_i, cnt);
  report(counts);
  return rc;
}
