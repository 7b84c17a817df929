// Op-counting build of the FP64 oracle (measurement infrastructure only).
//
// The oracle's own source, mppi_oracle.c, compiled as C++ with every binary64
// value replaced by Real, a wrapper around one double that counts each
// arithmetic operation applied to it.  The arithmetic and its order are the
// oracle's, so a count is the work of the plain definition of the method:
// the algorithmic operation count per rollout step that the throughput
// figures are priced with.  Counted per class:
//   add (additions and subtractions), mul, div, sqrt, transcendental (exp,
//   log, sin, cos, fmod), other (fabs, floor, comparisons: not flops).
// Structs of the counted build have the layout of the plain build (Real is
// one double), so the same ctypes structures drive both libraries.  Built
// without OpenMP: the counters are plain globals and every solve is serial.
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <cmath>
#include <type_traits>

namespace {
struct OpCounts {
    int64_t add, mul, div, sqrt, trans, other;
};
OpCounts g_ops = {0, 0, 0, 0, 0, 0};
}  // namespace

class Real {
public:
    Real() = default;
    Real(double x) : v_(x) {}  // literals and integers enter unconverted
    explicit operator double() const { return v_; }
    template <typename I, typename = typename std::enable_if<std::is_integral<I>::value>::type>
    explicit operator I() const { return (I)v_; }
    double raw() const { return v_; }

    Real &operator+=(Real o) { ++g_ops.add; v_ += o.v_; return *this; }
    Real &operator-=(Real o) { ++g_ops.add; v_ -= o.v_; return *this; }
    Real &operator*=(Real o) { ++g_ops.mul; v_ *= o.v_; return *this; }
    Real &operator/=(Real o) { ++g_ops.div; v_ /= o.v_; return *this; }
    Real operator-() const { return Real(-v_); }  // a sign flip, not an operation

    friend Real operator+(Real a, Real b) { ++g_ops.add; return Real(a.v_ + b.v_); }
    friend Real operator-(Real a, Real b) { ++g_ops.add; return Real(a.v_ - b.v_); }
    friend Real operator*(Real a, Real b) { ++g_ops.mul; return Real(a.v_ * b.v_); }
    friend Real operator/(Real a, Real b) { ++g_ops.div; return Real(a.v_ / b.v_); }
    friend bool operator<(Real a, Real b) { ++g_ops.other; return a.v_ < b.v_; }
    friend bool operator>(Real a, Real b) { ++g_ops.other; return a.v_ > b.v_; }
    friend bool operator<=(Real a, Real b) { ++g_ops.other; return a.v_ <= b.v_; }
    friend bool operator>=(Real a, Real b) { ++g_ops.other; return a.v_ >= b.v_; }
    friend bool operator==(Real a, Real b) { ++g_ops.other; return a.v_ == b.v_; }
    friend bool operator!=(Real a, Real b) { ++g_ops.other; return a.v_ != b.v_; }

private:
    double v_;
};
static_assert(sizeof(Real) == sizeof(double) && alignof(Real) == alignof(double), "layout of binary64");

static inline Real sqrt(Real a) { ++g_ops.sqrt; return Real(std::sqrt(a.raw())); }
static inline Real exp(Real a) { ++g_ops.trans; return Real(std::exp(a.raw())); }
static inline Real log(Real a) { ++g_ops.trans; return Real(std::log(a.raw())); }
static inline Real sin(Real a) { ++g_ops.trans; return Real(std::sin(a.raw())); }
static inline Real cos(Real a) { ++g_ops.trans; return Real(std::cos(a.raw())); }
static inline Real fmod(Real a, Real b) { ++g_ops.trans; return Real(std::fmod(a.raw(), b.raw())); }
static inline Real fabs(Real a) { ++g_ops.other; return Real(std::fabs(a.raw())); }
static inline Real floor(Real a) { ++g_ops.other; return Real(std::floor(a.raw())); }
static inline bool isfinite(Real a) { ++g_ops.other; return std::isfinite(a.raw()); }

// the oracle, with binary64 counted
#define double Real
#include "mppi_oracle.c"
#undef double

extern "C" {

void orc_ops_reset(void) { g_ops = OpCounts{0, 0, 0, 0, 0, 0}; }

// out: add, mul, div, sqrt, transcendental, other
void orc_ops_read(int64_t out[6])
{
    out[0] = g_ops.add;
    out[1] = g_ops.mul;
    out[2] = g_ops.div;
    out[3] = g_ops.sqrt;
    out[4] = g_ops.trans;
    out[5] = g_ops.other;
}

}  // extern "C"
