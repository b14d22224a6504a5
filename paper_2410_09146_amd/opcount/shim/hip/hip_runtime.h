// Host shim used only by the operation counter: the device math header is
// compiled with `double` replaced by a scalar type that tallies every FP64
// operation it performs.  Never part of the GPU build.
#pragma once
#include <cmath>
#include <cstdint>

#define GRMHD_OPCOUNT 1
#define __device__
#define __forceinline__ inline

struct OpCount { long long add = 0, mul = 0, div = 0, fma = 0, sqrt = 0, cmp = 0, tr = 0; };
extern OpCount g_ops;

struct cd {
  double v;
  constexpr cd() : v(0.0) {}
  constexpr cd(double x) : v(x) {}
  explicit operator int() const { return (int)v; }
};
inline cd operator+(cd a, cd b) { ++g_ops.add; return cd(a.v + b.v); }
inline cd operator-(cd a, cd b) { ++g_ops.add; return cd(a.v - b.v); }
inline cd operator*(cd a, cd b) { ++g_ops.mul; return cd(a.v * b.v); }
inline cd operator/(cd a, cd b) { ++g_ops.div; return cd(a.v / b.v); }
inline cd operator-(cd a) { return cd(-a.v); }
inline cd &operator+=(cd &a, cd b) { a = a + b; return a; }
inline cd &operator-=(cd &a, cd b) { a = a - b; return a; }
inline cd &operator*=(cd &a, cd b) { a = a * b; return a; }
inline cd &operator/=(cd &a, cd b) { a = a / b; return a; }
inline bool operator<(cd a, cd b) { ++g_ops.cmp; return a.v < b.v; }
inline bool operator>(cd a, cd b) { ++g_ops.cmp; return a.v > b.v; }
inline bool operator<=(cd a, cd b) { ++g_ops.cmp; return a.v <= b.v; }
inline bool operator>=(cd a, cd b) { ++g_ops.cmp; return a.v >= b.v; }
inline bool operator==(cd a, cd b) { ++g_ops.cmp; return a.v == b.v; }
inline cd sqrt(cd a) { ++g_ops.sqrt; return cd(std::sqrt(a.v)); }
inline cd fabs(cd a) { return cd(std::fabs(a.v)); }
inline cd fmin(cd a, cd b) { ++g_ops.cmp; return cd(std::fmin(a.v, b.v)); }
inline cd fmax(cd a, cd b) { ++g_ops.cmp; return cd(std::fmax(a.v, b.v)); }
inline cd fma(cd a, cd b, cd c) { ++g_ops.fma; return cd(std::fma(a.v, b.v, c.v)); }
inline bool isfinite(cd a) { return std::isfinite(a.v); }
// logarithms and exponentials (tabulated-EOS lookups) are tallied apart
inline cd exp(cd a) { ++g_ops.tr; return cd(std::exp(a.v)); }
inline cd log(cd a) { ++g_ops.tr; return cd(std::log(a.v)); }
// the hardware reciprocal estimate counts as the division it stands for
inline cd __builtin_amdgcn_rcp(cd a) { ++g_ops.div; return cd(1.0 / a.v); }

// vector and integer helpers the device header uses
struct double2 { cd x, y; };
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }

#define double cd
